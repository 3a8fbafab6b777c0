// C ABI of the hp space-time multigrid library (include/stmg.h): context
// set-up, device uploads, the V-cycle (Alg. 1 with Alg. 4-7) and FGMRES.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

#include "../../include/stmg.h"
#include "host.hpp"
#include "kernels.hpp"
#include "learned.hpp"

using namespace stmg;

namespace {

struct DeviceError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHK(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      throw DeviceError(std::string(#expr) + " failed: " + hipGetErrorString(e_));                \
  } while (0)

// tracked device allocations, freed with the context
struct Pool {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <typename T>
  T* alloc(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) throw Error(STMG_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    ptrs.push_back(p);
    bytes += n * sizeof(T);
    return static_cast<T*>(p);
  }
  template <typename T, typename S>
  T* upload(const std::vector<S>& v, hipStream_t s) {
    T* d = alloc<T>(v.size());
    if (v.empty()) return d;
    if constexpr (std::is_same<T, S>::value) {
      HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));  // the host vector may be a temporary
    } else {
      std::vector<T> c(v.begin(), v.end());
      HIPCHK(hipMemcpyAsync(d, c.data(), c.size() * sizeof(T), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    return d;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

template <typename T>
struct DevLevel {
  LevelArgs a{};
  int vform = STMG_VANKA_FACTORED;  // stored form of this level's local inverses
  T* tab = nullptr;
  T* geo = nullptr;  // Gauss-point geometry of the operator kernel
  T *Asw = nullptr, *Bm = nullptr, *F = nullptr, *Hinv = nullptr, *coef = nullptr, *dense = nullptr;
  T* E = nullptr;  // cell-local scratch of the Vanka correction
  T *b = nullptr, *x = nullptr, *r = nullptr;
  int64_t ndofs = 0;
};

template <typename T>
struct DevTransfer {
  TransferDev t{};
  T *P1 = nullptr, *P1T = nullptr, *E = nullptr, *Pt = nullptr;
  int *rlo = nullptr, *rhi = nullptr, *clo = nullptr, *chi = nullptr;
  T *tmp1 = nullptr, *tmp2 = nullptr, *tmp3 = nullptr;
};

template <typename T>
struct Hier {
  std::vector<DevLevel<T>> L;
  std::vector<DevTransfer<T>> X;
};

struct EventTimer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs;
  size_t used = 0;
  hipEvent_t a(hipStream_t s) {
    if (used == pairs.size()) {
      hipEvent_t e1, e2;
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventCreate(&e2));
      pairs.push_back({e1, e2});
    }
    HIPCHK(hipEventRecord(pairs[used].first, s));
    return pairs[used].first;
  }
  void b(hipStream_t s) {
    HIPCHK(hipEventRecord(pairs[used].second, s));
    ++used;
  }
  double total_s() {
    double t = 0;
    for (size_t i = 0; i < used; ++i) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, pairs[i].first, pairs[i].second));
      t += ms * 1e-3;
    }
    return t;
  }
  void reset() { used = 0; }
  ~EventTimer() {
    for (auto& p : pairs) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  }
};

}  // namespace

struct stmg_ctx {
  stmg_params p{};
  std::string err;
  hipStream_t stream = nullptr;
  Pool pool;
  std::vector<LevelHost> host;
  // FP64 view of every level (operator, per-op calls); FP32 hierarchy in mixed mode
  Hier<double> H64;
  Hier<float> H32;
  bool mixed = false;
  double *Cinv = nullptr, *Cg = nullptr;  // coarsest level: bordered subinterval inverse, coupling
  int64_t nd_coarse = 0;
  double* mom0 = nullptr;  // finest-level pressure moments
  double volume0 = 1.0;
  // FGMRES work
  double *V = nullptr, *Z = nullptr, *w = nullptr, *u = nullptr, *partial = nullptr, *dh = nullptr,
         *dtmp = nullptr;
  float* Z32 = nullptr;    // mixed precision: the preconditioned basis, as the FP32 V-cycle leaves it
  double* zt = nullptr;    // mixed precision: FP64 copy of the current basis vector
  int cap = 0;
  std::vector<double> history;
  bool phase_timing = false;
  EventTimer t_smooth, t_vcyc, t_op;
  // learned correction
  NetDev net;
  bool net_ready = false, learned_on = false, learned_disabled = false;
  int learned_steps = 0;  // corrections applied in the current solve
  int learned_reading = 1;  // 1: every level reaching a Q2/P1 x DG(1) level on its mesh; 2: those levels only
  std::vector<void*> lsave;  // per level: copy of x before a correction
  // time marching: right-hand side and Dirichlet values of the current slab
  double *slab_b = nullptr, *slab_g = nullptr;
  // execution options (stmg_set_option)
  int opt_apply_nper = 0;      // subintervals per wave of the operator's cell kernel (0: automatic)
  int opt_apply_variant = 0;   // loop order of the operator's cell kernel (0: automatic)
  int64_t opt_net_chunk = 0;   // space-time cells per inference chunk (0: the default)
  int64_t opt_inject_nonfinite = 0;  // test hook: preconditioner application whose output is made NaN
};

namespace {

LevelArgs level_args(const LevelHost& L) {
  // the kernels index cells, nodes and pressure dofs of one field in 32 bits
  if (L.nodes >= (int64_t(1) << 31) || L.Mp >= (int64_t(1) << 31))
    throw Error(STMG_EUNSUPPORTED, "level with 2^31 or more nodes or pressure dofs per field");
  LevelArgs a;
  a.d = L.d; a.n = L.n; a.q = L.q; a.Q = L.Q; a.nn = L.nn; a.nt = L.nt; a.C = L.C; a.N = L.N; a.nloc = L.nloc;
  a.nodes = L.nodes; a.Mv = L.Mv; a.Mp = L.Mp; a.slab = L.slab;
  return a;
}

std::vector<double> pack_tables(const LevelHost& L) {
  std::vector<double> t;
  const SpaceTables& S = L.st;
  t.insert(t.end(), S.S.begin(), S.S.end());
  t.insert(t.end(), S.Dg.begin(), S.Dg.end());
  t.insert(t.end(), S.gx.begin(), S.gx.end());
  t.insert(t.end(), S.gw.begin(), S.gw.end());
  t.insert(t.end(), L.td.K.begin(), L.td.K.end());
  t.insert(t.end(), L.td.phim1.begin(), L.td.phim1.end());
  for (int a = 0; a < L.nt; ++a) t.push_back(0.5 * L.tau * L.td.w[a]);
  t.insert(t.end(), S.psi.begin(), S.psi.end());
  return t;
}

// The stored form of a level's local inverses: the requested one, or for
// STMG_VANKA_AUTO the one measured faster at that element (the decoupled form
// halves the bytes of the dominant factor, which pays on levels with 64 and
// more velocity nodes per cell; below, the per-cell fixed costs dominate and
// the Schur-factored kernel is faster).
constexpr int kFormDiagonal = 4;  // the diagonal Vanka (decoupled, diagonal spatial blocks)

int vanka_form(const stmg_params& p, const LevelHost& L) {
  if (p.local_solver == STMG_LOCAL_DIAGONAL) return kFormDiagonal;
  if (p.vanka_mode != STMG_VANKA_AUTO) return p.vanka_mode;
  return L.nloc >= 64 ? STMG_VANKA_DECOUPLED : STMG_VANKA_FACTORED;
}

template <typename T>
void build_hier(stmg_ctx* c, Hier<T>& H, const std::vector<VankaFactors>& VF,
                const std::vector<std::vector<double>>& dense, const std::vector<VankaDecoupled>& VD,
                bool with_vanka) {
  hipStream_t s = c->stream;
  const size_t nlev = c->host.size();
  H.L.resize(nlev);
  for (size_t l = 0; l < nlev; ++l) {
    const LevelHost& L = c->host[l];
    DevLevel<T>& D = H.L[l];
    D.a = level_args(L);
    D.vform = vanka_form(c->p, L);
    D.tab = c->pool.upload<T>(pack_tables(L), s);
    {
      std::vector<double> g;
      apply_geometry(L, g);
      D.geo = c->pool.upload<T>(g, s);
    }
    D.ndofs = L.ndofs;
    // cell-local scratch shared by the operator and the smoother of this level
    D.E = c->pool.alloc<T>((size_t)L.ncells * L.d * L.nt * L.nloc * L.N);
    D.b = c->pool.alloc<T>(L.ndofs);
    D.x = c->pool.alloc<T>(L.ndofs);
    D.r = c->pool.alloc<T>(L.ndofs);
    if (with_vanka && l + 1 < nlev && D.vform == kFormDiagonal) {
      const VankaDecoupled& V = VD[l];
      const int J = V.te.J, nt = L.nt, nl = L.nloc, C = L.C;
      const int R4 = vanka_tdec_row(C);
      if (V.te.nreal != nt % 2 || J != (nt + 1) / 2)
        throw Error(STMG_EUNSUPPORTED, "unexpected eigenvalue structure of the temporal matrix");
      std::vector<double> tw;
      for (const auto& z : V.te.T) { tw.push_back(z.real()); tw.push_back(z.imag()); }
      for (const auto& z : V.te.Wt) { tw.push_back(z.real()); tw.push_back(z.imag()); }
      D.coef = c->pool.upload<T>(tw, s);
      std::vector<T> Dw((size_t)L.ncells * J * nl * 2), Hr((size_t)L.ncells * J * C * R4, T(0));
      for (size_t i = 0; i < V.Dinv.size(); ++i) {
        Dw[2 * i] = (T)V.Dinv[i].real();
        Dw[2 * i + 1] = (T)V.Dinv[i].imag();
      }
      for (int64_t cl = 0; cl < L.ncells; ++cl)
        for (int j = 0; j < J; ++j) {
          const std::complex<double>* Hi = &V.Hinv[((size_t)cl * J + j) * C * C];
          for (int l = 0; l < C; ++l)
            for (int l2 = 0; l2 < C; ++l2) {
              T* h = &Hr[(((size_t)cl * J + j) * C + l) * R4 + 2 * l2];
              h[0] = (T)Hi[(size_t)l * C + l2].real();
              h[1] = (T)Hi[(size_t)l * C + l2].imag();
            }
        }
      D.Asw = c->pool.upload<T>(Dw, s);
      D.Bm = c->pool.upload<T>(V.Bm, s);
      D.Hinv = c->pool.upload<T>(Hr, s);
    } else if (with_vanka && l + 1 < nlev && D.vform == STMG_VANKA_DECOUPLED) {
      const VankaDecoupled& V = VD[l];
      const int J = V.te.J, nt = L.nt, nl = L.nloc, C = L.C, d = L.d;
      const int mp = (nl + 15) & ~15, R4 = vanka_tdec_row(C);
      if (V.te.nreal != nt % 2 || J != (nt + 1) / 2)
        throw Error(STMG_EUNSUPPORTED, "unexpected eigenvalue structure of the temporal matrix");
      // per level: T (J x nt) then Wt (nt x J), complex as (re, im)
      std::vector<double> tw;
      for (const auto& z : V.te.T) { tw.push_back(z.real()); tw.push_back(z.imag()); }
      for (const auto& z : V.te.Wt) { tw.push_back(z.real()); tw.push_back(z.imag()); }
      D.coef = c->pool.upload<T>(tw, s);
      const int64_t aw = vanka_tdec_aw(nl, nt), half = aw / nt;  // half: one real block's tiles
      std::vector<T> A((size_t)L.ncells * aw, T(0));
      std::vector<T> Fr((size_t)L.ncells * J * d * nl * R4, T(0)), Hr((size_t)L.ncells * J * C * R4, T(0));
      int asym = 0;  // blocks whose inverse is not symmetric to rounding
#pragma omp parallel for schedule(static) reduction(+ : asym)
      for (int64_t cl = 0; cl < L.ncells; ++cl) {
        for (int j = 0; j < J; ++j) {
          const bool cpx = j >= V.te.nreal;
          T* X = &A[(size_t)cl * aw + (size_t)(j < V.te.nreal ? j : 2 * j - V.te.nreal) * half];
          const std::complex<double>* Ai = &V.Ainv[((size_t)cl * J + j) * nl * nl];
          // the upper tiles of the symmetric part.  Ainv_j is symmetric in
          // exact arithmetic, and its computed asymmetry is the inversion's
          // rounding, so symmetrizing costs no accuracy; the check below only
          // catches a block that is not symmetric at all (a construction
          // error), with room for blocks with condition numbers up to ~1e9
          double amax = 0.0, dmax = 0.0;
          for (int row = 0; row < nl; ++row)
            for (int k = 0; k < nl; ++k) {
              const std::complex<double> z = Ai[(size_t)row * nl + k], zt = Ai[(size_t)k * nl + row];
              amax = std::max(amax, std::abs(z));
              dmax = std::max(dmax, std::abs(z - zt));
              if (row / 16 > k / 16) continue;
              const std::complex<double> zs = 0.5 * (z + zt);
              X[vanka_sym_index(mp, row, k)] = (T)zs.real();
              if (cpx) X[half + vanka_sym_index(mp, row, k)] = (T)zs.imag();
            }
          if (!(dmax <= 1e-6 * amax)) ++asym;
          const std::complex<double>* F = &V.F[((size_t)cl * J + j) * d * nl * C];
          for (int ci = 0; ci < d * nl; ++ci)
            for (int l = 0; l < C; ++l) {
              T* f = &Fr[(((size_t)cl * J + j) * d * nl + ci) * R4 + 2 * l];
              f[0] = (T)F[(size_t)ci * C + l].real();
              f[1] = (T)F[(size_t)ci * C + l].imag();
            }
          const std::complex<double>* Hi = &V.Hinv[((size_t)cl * J + j) * C * C];
          for (int l = 0; l < C; ++l)
            for (int l2 = 0; l2 < C; ++l2) {
              T* h = &Hr[(((size_t)cl * J + j) * C + l) * R4 + 2 * l2];
              h[0] = (T)Hi[(size_t)l * C + l2].real();
              h[1] = (T)Hi[(size_t)l * C + l2].imag();
            }
        }
      }
      if (asym) throw Error(STMG_EUNSUPPORTED, "a decoupled local velocity inverse is not symmetric");
      D.Asw = c->pool.upload<T>(A, s);
      D.Bm = c->pool.upload<T>(V.Bm, s);
      D.F = c->pool.upload<T>(Fr, s);
      D.Hinv = c->pool.upload<T>(Hr, s);
    } else if (with_vanka && l + 1 < nlev) {
      const VankaFactors& V = VF[l];
      D.coef = c->pool.upload<T>(V.coef, s);
      if (D.vform == STMG_VANKA_DENSE) {
        D.dense = c->pool.upload<T>(dense[l], s);
      } else {
        // A_s^{-1} in MFMA operand order, padded to a multiple of 16
        const int m = V.m, mp = (m + 15) & ~15;
        std::vector<T> sw((size_t)L.ncells * mp * mp, T(0));
        for (int64_t cl = 0; cl < L.ncells; ++cl)
          for (int k = 0; k < m; ++k)
            for (int row = 0; row < m; ++row)
              sw[(size_t)cl * mp * mp + vanka_swizzle_index(mp, row, k)] =
                  (T)V.As_inv[((size_t)cl * m + k) * m + row];
        D.Asw = c->pool.upload<T>(sw, s);
        D.Bm = c->pool.upload<T>(V.Bm, s);
        // F and H^{-1} row by row (each row padded to a multiple of 4 values),
        // so that a thread reads a row with 16-byte loads
        const int P = V.P, P4 = vanka_row_pad(P);
        std::vector<T> Fr((size_t)L.ncells * L.d * m * P4, T(0)), Hr((size_t)L.ncells * P * P4, T(0));
        for (int64_t cl = 0; cl < L.ncells; ++cl) {
          for (int comp = 0; comp < L.d; ++comp)
            for (int q = 0; q < P; ++q)
              for (int row = 0; row < m; ++row)
                Fr[(((size_t)cl * L.d + comp) * m + row) * P4 + q] =
                    (T)V.F[(((size_t)cl * L.d + comp) * P + q) * m + row];
          for (int q = 0; q < P; ++q)
            for (int pp = 0; pp < P; ++pp)
              Hr[((size_t)cl * P + pp) * P4 + q] = (T)V.Hinv[((size_t)cl * P + q) * P + pp];
        }
        D.F = c->pool.upload<T>(Fr, s);
        D.Hinv = c->pool.upload<T>(Hr, s);
      }
    }
  }
  H.X.resize(nlev - 1);
  for (size_t l = 0; l + 1 < nlev; ++l) {
    const LevelHost& F = c->host[l];
    const LevelHost& C = c->host[l + 1];
    Transfer T0 = build_transfer(F, C);
    DevTransfer<T>& X = H.X[l];
    X.t.nnf = T0.nnf; X.t.nnc = T0.nnc; X.t.npos = T0.npos; X.t.ntf = T0.ntf; X.t.ntc = T0.ntc;
    X.t.time_change = T0.time_change;

    std::vector<double> P1T((size_t)T0.nnc * T0.nnf);
    for (int g = 0; g < T0.nnf; ++g)
      for (int h = 0; h < T0.nnc; ++h) P1T[(size_t)h * T0.nnf + g] = T0.P1[(size_t)g * T0.nnc + h];
    X.t.max_row_p1 = X.t.max_row_p1t = 0;
    for (int g = 0; g < T0.nnf; ++g) X.t.max_row_p1 = std::max(X.t.max_row_p1, T0.row_hi[g] - T0.row_lo[g]);
    for (int h = 0; h < T0.nnc; ++h) X.t.max_row_p1t = std::max(X.t.max_row_p1t, T0.col_hi[h] - T0.col_lo[h]);
    if (X.t.max_row_p1 > 16 || X.t.max_row_p1t > 16)
      throw Error(STMG_EUNSUPPORTED, "transfer rows longer than 16 taps");
    std::vector<int> brk;
    X.t.vt_p1 = vtransfer_plan(T0.row_lo, T0.row_hi, F.d, X.t.max_row_p1, false, sizeof(T), X.t.cap_p1, brk);
    if (X.t.vt_p1) X.t.brk_p1 = c->pool.upload<int>(brk, s);
    X.t.vt_p1t = vtransfer_plan(T0.col_lo, T0.col_hi, F.d, X.t.max_row_p1t, true, sizeof(T), X.t.cap_p1t, brk);
    if (X.t.vt_p1t) X.t.brk_p1t = c->pool.upload<int>(brk, s);
    // banded, transposed: Mb[u][row] = M[row][lo(row) + u], u < 16 (zero past the row)
    std::vector<double> P1b((size_t)16 * T0.nnf, 0.0), P1Tb((size_t)16 * T0.nnc, 0.0);
    for (int g = 0; g < T0.nnf; ++g)
      for (int u = 0; u < T0.row_hi[g] - T0.row_lo[g]; ++u)
        P1b[(size_t)u * T0.nnf + g] = T0.P1[(size_t)g * T0.nnc + T0.row_lo[g] + u];
    for (int h = 0; h < T0.nnc; ++h)
      for (int u = 0; u < T0.col_hi[h] - T0.col_lo[h]; ++u)
        P1Tb[(size_t)u * T0.nnc + h] = P1T[(size_t)h * T0.nnf + T0.col_lo[h] + u];
    X.P1 = c->pool.upload<T>(P1b, s);
    X.P1T = c->pool.upload<T>(P1Tb, s);
    X.rlo = c->pool.upload<int>(T0.row_lo, s);
    X.rhi = c->pool.upload<int>(T0.row_hi, s);
    X.clo = c->pool.upload<int>(T0.col_lo, s);
    X.chi = c->pool.upload<int>(T0.col_hi, s);
    X.E = c->pool.upload<T>(T0.E, s);
    X.Pt = c->pool.upload<T>(T0.Pt, s);
    // temporaries: batches of d-dimensional node arrays at fine time resolution
    int64_t nb = (int64_t)F.N * F.nt * F.d;
    int64_t big = std::max<int64_t>(F.nn, C.nn);
    int64_t per = F.d == 3 ? big * big * big : big * big;
    X.tmp1 = c->pool.alloc<T>(nb * per);
    X.tmp2 = c->pool.alloc<T>(nb * per);
    X.tmp3 = c->pool.alloc<T>((int64_t)F.N * F.nt * (C.Mv + C.Mp));
  }
  HIPCHK(hipStreamSynchronize(s));
}

// ------------------------------------------------------------- level ops
template <typename T>
void op_apply(stmg_ctx* c, DevLevel<T>& D, const T* x, const T* b, T* y, int mode) {
  HIPCHK(launch_apply<T>(D.a, D.geo, D.tab, x, b, y, mode, D.E, c->stream, true, c->opt_apply_nper,
                         c->opt_apply_variant));
}

// E: the cell-local scratch of the velocity corrections (the level's own, or
// the allocation-free entry point's)
template <typename T>
void op_vanka_with(stmg_ctx* c, DevLevel<T>& D, const T* r, T* x, T* E, bool xzero) {
  // xzero: x holds no values yet and starts at 0
  T om = (T)c->p.omega;
  if (D.vform == STMG_VANKA_DENSE) {
    if (xzero) HIPCHK(launch_fill<T>(x, T(0), D.ndofs, c->stream));
    HIPCHK(launch_vanka_dense<T>(D.a, D.dense, r, x, om, c->stream));
  } else if (D.vform == STMG_VANKA_DECOUPLED || D.vform == kFormDiagonal) {
    HIPCHK(launch_vanka_decoupled<T>(D.a, D.Asw, D.Bm, D.F, D.Hinv, D.coef, r, x, om, E, c->stream, true, xzero,
                                     D.vform == kFormDiagonal));
  } else {
    HIPCHK(launch_vanka_factored<T>(D.a, D.Asw, D.Bm, D.F, D.Hinv, D.coef, r, x, om, E, c->stream, true, xzero));
  }
}

template <typename T>
void op_vanka(stmg_ctx* c, DevLevel<T>& D, const T* r, T* x, bool xzero = false) {
  op_vanka_with<T>(c, D, r, x, D.E, xzero);
}

template <typename T>
bool learned_step(stmg_ctx* c, DevLevel<T>& D, int level, const T* b, T* x);

// zero_start: x starts at 0 (its contents are ignored; with steps == 0 it is set to 0).
// Returns whether D.r holds b - S x on exit (left there by a learned step).
template <typename T>
bool op_smooth(stmg_ctx* c, DevLevel<T>& D, const T* b, T* x, int steps, bool zero_start, int level = -1) {
  if (zero_start && steps == 0) HIPCHK(launch_fill<T>(x, T(0), D.ndofs, c->stream));
  bool r_current = false;
  for (int s = 0; s < steps; ++s) {
    const T* r = b;
    if (!(zero_start && s == 0)) {
      if (!r_current) op_apply<T>(c, D, x, b, D.r, 1);
      r = D.r;
    }
    if (c->phase_timing) c->t_smooth.a(c->stream);
    op_vanka<T>(c, D, r, x, zero_start && s == 0);
    if (c->phase_timing) c->t_smooth.b(c->stream);
    r_current = level >= 0 && learned_step<T>(c, D, level, b, x);
  }
  return r_current;
}

template <typename T>
void op_restrict(stmg_ctx* c, Hier<T>& H, int l, const T* fine, T* coarse) {
  DevTransfer<T>& X = H.X[l];
  HIPCHK(launch_restrict<T>(H.L[l].a, H.L[l + 1].a, X.t, X.P1T, X.clo, X.chi, X.E, X.Pt, fine, coarse, X.tmp1,
                            X.tmp2, X.tmp3, c->stream));
}

template <typename T>
void op_prolongate_add(stmg_ctx* c, Hier<T>& H, int l, const T* coarse, T* fine) {
  DevTransfer<T>& X = H.X[l];
  HIPCHK(launch_prolongate_add<T>(H.L[l].a, H.L[l + 1].a, X.t, X.P1, X.rlo, X.rhi, X.E, X.Pt, coarse, fine, X.tmp1,
                                  X.tmp2, X.tmp3, c->stream));
}

// ------------------------------------------------------------- learned
constexpr int64_t kNetChunk = 65536;  // samples per inference chunk

void net_alloc(stmg_ctx* c, int64_t batch) {
  NetDev& N = c->net;
  if (!c->net_ready) {
    N.w = c->pool.alloc<float>(kNetParams);
    N.m = c->pool.alloc<float>(kNetParams);
    N.v = c->pool.alloc<float>(kNetParams);
    N.g = c->pool.alloc<float>(kNetParams);
    N.fw = c->pool.alloc<uint16_t>(27 * (16 * 32 + 32 * 32 + 32 * 16));
    N.bw = c->pool.alloc<uint16_t>(27 * (16 * 32 + 32 * 32));
    N.cap = kNetChunk;
    N.x = c->pool.alloc<uint16_t>(N.cap * 512);
    N.h1 = c->pool.alloc<uint16_t>(N.cap * 1024);
    N.h2 = c->pool.alloc<uint16_t>(N.cap * 1024);
    N.y = c->pool.alloc<float>(N.cap * 512);
    N.dy = c->pool.alloc<uint16_t>(N.cap * 512);
    N.scale = c->pool.alloc<float>(N.cap);
    N.mask = c->pool.alloc<float>(N.cap * 27);
    N.tv = c->pool.alloc<float>(N.cap * 162);
    N.tp = c->pool.alloc<float>(N.cap * 8);
    N.red = c->pool.alloc<double>(2 * N.cap + 8);
    HIPCHK(launch_fill<float>(N.m, 0.0f, kNetParams, c->stream));
    HIPCHK(launch_fill<float>(N.v, 0.0f, kNetParams, c->stream));
    c->net_ready = true;
  }
  int64_t nb = (std::min<int64_t>(batch, N.cap) + 7) / 8;
  if (nb > N.pcap) {
    N.partial = c->pool.alloc<float>((size_t)nb * kNetParams);
    N.pcap = nb;
  }
}

bool net_level(const LevelArgs& a) { return a.d == 3 && a.Q == 3 && a.nt == 2; }

// How the learned correction reaches level l: 1 the level has the network's
// element; 2 the next coarser level has it, on the same mesh and the same
// subintervals (the correction is computed there: residual restricted,
// network correction prolongated); 0 not at all.
int net_route(const stmg_ctx* c, int l) {
  const auto& L = c->H64.L;
  if (net_level(L[l].a)) return 1;
  if (l + 1 < (int)L.size() && net_level(L[l + 1].a) && L[l + 1].a.n == L[l].a.n && L[l + 1].a.N == L[l].a.N)
    return 2;
  return 0;
}

template <typename T>
Hier<T>& hier_of(stmg_ctx* c);
template <>
Hier<double>& hier_of<double>(stmg_ctx* c) { return c->H64; }
template <>
Hier<float>& hier_of<float>(stmg_ctx* c) { return c->H32; }

// x = net(r) on level D (zero_start: x holds no values yet), or x += net(r):
// velocity into E, then gathered with weight 1; pressure written or added
template <typename T>
void net_correct(stmg_ctx* c, DevLevel<T>& D, const T* r, T* x, bool zero_start) {
  const int64_t total = (int64_t)D.a.N * (D.a.Mp / D.a.C);
  const int64_t chunk = c->opt_net_chunk > 0 ? std::min<int64_t>(c->opt_net_chunk, kNetChunk) : kNetChunk;
  for (int64_t first = 0; first < total; first += chunk) {
    int64_t cnt = std::min<int64_t>(chunk, total - first);
    HIPCHK(net_inputs<T>(D.a, c->net, r, (const T*)nullptr, first, cnt, c->stream));
    HIPCHK(net_forward(c->net, cnt, c->stream, false));
    HIPCHK(net_correction<T>(D.a, c->net, first, cnt, D.E, x, c->stream, zero_start));
  }
  HIPCHK(launch_vanka_gather_only<T>(D.a, D.E, x, T(1), c->stream, zero_start));
}

template <typename T>
double norm2(stmg_ctx* c, const T* v, int64_t n);

// After a Vanka sweep: r = b - S x, c = net(r), w = S c and x += alpha c with
// the residual-minimising alpha = <r, w> / <w, w>, so the level residual
// cannot grow.  If the direction does not reduce it enough (below) the
// correction is skipped and switched off for the rest of the solve.
// cv = the network correction of the residual r on level l (route 1), or
// P net(P^T r) through the next level (route 2), with the next level's
// learned work vectors as temporaries
template <typename T>
void learned_correction_at(stmg_ctx* c, int level, int route, const T* r, T* cv) {
  Hier<T>& H = hier_of<T>(c);
  DevLevel<T>& D = H.L[level];
  if (route == 1) {
    net_correct<T>(c, D, r, cv, true);
    return;
  }
  HIPCHK(launch_fill<T>(cv, T(0), D.ndofs, c->stream));
  DevLevel<T>& Cl = H.L[level + 1];
  T* rc = static_cast<T*>(c->lsave[2 * (level + 1)]);
  T* cc = static_cast<T*>(c->lsave[2 * (level + 1) + 1]);
  op_restrict<T>(c, H, level, r, rc);
  net_correct<T>(c, Cl, rc, cc, true);
  op_prolongate_add<T>(c, H, level, cc, cv);
}

// Smallest fraction of |r|^2 a learned step must remove to stay switched on.
constexpr double kLearnedMinGain = 0.02;

// Returns whether it ran: then D.r holds b - S x for the x it leaves (the
// residual after the update is r - alpha w, so the caller need not apply S again).
template <typename T>
bool learned_step(stmg_ctx* c, DevLevel<T>& D, int level, const T* b, T* x) {
  if (!c->learned_on || c->learned_disabled || !c->net_ready) return false;
  const int route = net_route(c, level);
  if (route == 0 || (route == 2 && c->learned_reading != 1)) return false;
  T* cv = static_cast<T*>(c->lsave[2 * level]);
  T* wv = static_cast<T*>(c->lsave[2 * level + 1]);
  op_apply<T>(c, D, x, b, D.r, 1);
  learned_correction_at<T>(c, level, route, D.r, cv);
  op_apply<T>(c, D, cv, cv, wv, 0);
  double d3[3];  // <r, w>, <w, w>, <r, r>: one reduction, one host synchronisation
  HIPCHK(launch_dot3<T>(D.r, wv, D.ndofs, c->partial, c->dh, c->stream));
  HIPCHK(hipMemcpyAsync(d3, c->dh, sizeof(d3), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const double rw = d3[0], ww = d3[1], rr = d3[2];
  // the step lowers |r|^2 by the fraction rw^2 / (ww rr); below kLearnedMinGain
  // it is not worth the network's cost, and a step that cannot lower it at
  // all (rw <= 0, non-finite) would raise the residual
  if (!(rw > 0.0) || !(ww > 0.0) || !std::isfinite(rw / ww) || !(rw * (rw / ww) >= kLearnedMinGain * rr)) {
    c->learned_disabled = true;
    return true;  // x unchanged: D.r = b - S x
  }
  const T alpha = (T)(rw / ww);
  ++c->learned_steps;
  HIPCHK(launch_axpy<T>(x, alpha, cv, D.ndofs, c->stream));
  HIPCHK(launch_axpy<T>(D.r, -alpha, wv, D.ndofs, c->stream));
  return true;
}

// x_l = V(b_l) on level l (zero initial guess), Alg. 1.
template <typename T>
void vcycle(stmg_ctx* c, Hier<T>& H, int l) {
  DevLevel<T>& D = H.L[l];
  const int last = (int)H.L.size() - 1;
  if (l == last) {
    HIPCHK(launch_coarse<T>(D.a.slab, D.a.Mv, D.a.nt, D.a.N, c->Cinv, c->Cg, D.b, D.x, c->stream));
    return;
  }
  if (!op_smooth<T>(c, D, D.b, D.x, c->p.nu_pre, true, l))               // presmoothing from x = 0
    op_apply<T>(c, D, D.x, D.b, D.r, 1);                                 // residual (unless left there)
  op_restrict<T>(c, H, l, D.r, H.L[l + 1].b);                            // restriction
  vcycle<T>(c, H, l + 1);                                                // coarse-grid correction
  op_prolongate_add<T>(c, H, l, H.L[l + 1].x, D.x);                      // prolongation and correction
  op_smooth<T>(c, D, D.b, D.x, c->p.nu_post, false, l);                  // postsmoothing
}

// Mixed precision: z = V(b) with the finest FP32 level's b already holding
// the input; the V-cycle writes its result straight into z (FP32).
void precondition_f32(stmg_ctx* c, float* z) {
  DevLevel<float>& D = c->H32.L[0];
  struct Restore {
    float*& x;
    float* keep;
    ~Restore() { x = keep; }
  } restore{D.x, D.x};
  if (c->phase_timing) c->t_vcyc.a(c->stream);
  D.x = z;
  vcycle<float>(c, c->H32, 0);
  if (c->phase_timing) c->t_vcyc.b(c->stream);
}

// z = V(v) for FP64 vectors v, z (device), in the context's precision
void precondition(stmg_ctx* c, const double* v, double* z) {
  if (c->phase_timing) c->t_vcyc.a(c->stream);
  if (c->mixed) {
    DevLevel<float>& D = c->H32.L[0];
    HIPCHK(launch_cast_d2f(v, D.b, D.ndofs, c->stream));
    vcycle<float>(c, c->H32, 0);
    HIPCHK(launch_cast_f2d(D.x, z, D.ndofs, c->stream));
  } else {
    DevLevel<double>& D = c->H64.L[0];
    if (v != z) {
      // the V-cycle reads the finest level's b and writes its x: run it on v
      // and z themselves (b is only read on the finest level)
      struct Restore {
        double*& b;
        double*& x;
        double* kb;
        double* kx;
        ~Restore() {
          b = kb;
          x = kx;
        }
      } restore{D.b, D.x, D.b, D.x};
      D.b = const_cast<double*>(v);
      D.x = z;
      vcycle<double>(c, c->H64, 0);
    } else {
      HIPCHK(hipMemcpyAsync(D.b, v, D.ndofs * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      vcycle<double>(c, c->H64, 0);
      HIPCHK(hipMemcpyAsync(z, D.x, D.ndofs * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
  }
  if (c->phase_timing) c->t_vcyc.b(c->stream);
}

int fail(stmg_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

template <typename F>
int guarded(stmg_ctx* c, F&& f) {
  try {
    if (c) HIPCHK(hipSetDevice(c->p.device));
    f();
    return STMG_OK;
  } catch (const Error& e) {
    return fail(c, e.code, e.what());
  } catch (const DeviceError& e) {
    return fail(c, STMG_EDEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(c, STMG_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, STMG_EINVAL, e.what());
  }
}

double dot(stmg_ctx* c, const double* a, const double* b, int64_t n) {
  HIPCHK(launch_multidot(a, n, 1, b, n, c->partial, c->dh, c->stream));
  double h;
  HIPCHK(hipMemcpyAsync(&h, c->dh, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return h;
}

template <typename T>
double norm2(stmg_ctx* c, const T* v, int64_t n) {
  if constexpr (std::is_same<T, double>::value) {
    return std::sqrt(dot(c, v, v, n));
  } else {
    HIPCHK(launch_cast_f2d(v, c->dtmp, n, c->stream));
    return std::sqrt(dot(c, c->dtmp, c->dtmp, n));
  }
}

bool valid_pow2(int v) { return v >= 1 && (v & (v - 1)) == 0; }

}  // namespace

// Run a level operation in the context's precision on FP64 user vectors.
template <typename F64, typename F32>
static int per_op(stmg_ctx* c, F64&& f64, F32&& f32) {
  return guarded(c, [&] {
    if (c->mixed) f32();
    else f64();
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

// ======================================================================= ABI
extern "C" {

stmg_status stmg_default_params(stmg_params* p) {
  if (!p) return STMG_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->dim = 3; p->n_cells_1d = 4; p->n_coarse_1d = 2; p->deform_amp = 0.0;
  p->r = 1; p->k = 1; p->n_sub = 2; p->tau = 0.05; p->nu = 1.0;
  p->r_min = 1; p->k_min = 1; p->time_h_coarsening = 0; p->placement = 0; p->nu_pre = 1; p->nu_post = 1; p->omega = 0.8;
  p->precision = STMG_FP64; p->vanka_mode = STMG_VANKA_AUTO; p->device = 0; p->stream = nullptr;
  return STMG_OK;
}

static int check_params(const stmg_params* p, std::string& msg) {
  if (!p) { msg = "null params"; return STMG_EINVAL; }
  if (p->dim != 2 && p->dim != 3) { msg = "dim must be 2 or 3"; return STMG_EINVAL; }
  if (p->n_coarse_1d < 1 || p->n_cells_1d < p->n_coarse_1d || p->n_cells_1d % p->n_coarse_1d != 0 ||
      !valid_pow2(p->n_cells_1d / p->n_coarse_1d)) {
    msg = "n_cells_1d must be n_coarse_1d times a power of two"; return STMG_EINVAL;
  }
  if (!valid_pow2(p->n_sub) || p->n_sub > 8) { msg = "n_sub must be 1, 2, 4 or 8"; return STMG_EINVAL; }
  if (p->r < 1 || p->r > 2 || p->r_min < 1 || p->r_min > p->r) { msg = "supported: 1 <= r_min <= r <= 2"; return STMG_EUNSUPPORTED; }
  if (p->k < 0 || p->k > 3 || p->k_min < 0 || p->k_min > p->k) { msg = "supported: 0 <= k_min <= k <= 3"; return STMG_EUNSUPPORTED; }
  if (!(p->tau > 0) || !(p->nu > 0 || p->nu_fn)) { msg = "tau and nu must be positive"; return STMG_EINVAL; }
  if (!(p->omega > 0) || p->nu_pre < 0 || p->nu_post < 0) { msg = "bad smoother parameters"; return STMG_EINVAL; }
  if (p->precision != STMG_FP64 && p->precision != STMG_MIXED_FP32) { msg = "bad precision"; return STMG_EINVAL; }
  if (p->vanka_mode < STMG_VANKA_FACTORED || p->vanka_mode > STMG_VANKA_AUTO) { msg = "bad vanka_mode"; return STMG_EINVAL; }
  if (p->local_solver != STMG_LOCAL_EXACT && p->local_solver != STMG_LOCAL_DIAGONAL) { msg = "bad local_solver"; return STMG_EINVAL; }
  if (p->placement != 0 && p->placement != 1) { msg = "bad placement"; return STMG_EINVAL; }
  return STMG_OK;
}

stmg_status stmg_hierarchy(const stmg_params* p, int max_levels, int* levels_out, int* n_levels) {
  std::string msg;
  int e = check_params(p, msg);
  if (e) return (stmg_status)e;
  if (!levels_out || !n_levels) return STMG_EINVAL;
  auto L = build_levels(p->n_cells_1d, p->r, p->k, p->n_sub, p->n_coarse_1d, p->r_min, p->k_min,
                        p->time_h_coarsening != 0, p->placement);
  *n_levels = (int)L.size();
  for (int i = 0; i < (int)L.size() && i < max_levels; ++i) {
    levels_out[4 * i + 0] = L[i].n; levels_out[4 * i + 1] = L[i].r;
    levels_out[4 * i + 2] = L[i].k; levels_out[4 * i + 3] = L[i].N;
  }
  return STMG_OK;
}

stmg_status stmg_setup(const stmg_params* p, stmg_ctx** out) {
  if (!out) return STMG_EINVAL;
  *out = nullptr;
  std::string msg;
  int e = check_params(p, msg);
  if (e) return (stmg_status)e;
  auto* c = new (std::nothrow) stmg_ctx();
  if (!c) return STMG_ENOMEM;
  c->p = *p;
  c->mixed = p->precision == STMG_MIXED_FP32;
  int rc = guarded(c, [&] {
    c->stream = static_cast<hipStream_t>(p->stream);
    Params P;
    P.d = p->dim; P.n = p->n_cells_1d; P.n_coarse = p->n_coarse_1d; P.r = p->r; P.k = p->k; P.N = p->n_sub;
    P.r_min = p->r_min; P.k_min = p->k_min; P.time_h = p->time_h_coarsening != 0; P.placement = p->placement;
    P.amp = p->deform_amp; P.tau = p->tau; P.nu = p->nu;
    if (p->nu_fn) {
      stmg_nu_fn fn = p->nu_fn;
      void* user = p->nu_user;
      P.nu_fn = [fn, user](int n, const double* xyz, double* o) { fn(n, xyz, o, user); };
    }
    auto specs = build_levels(P.n, P.r, P.k, P.N, P.n_coarse, P.r_min, P.k_min, P.time_h, P.placement);
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    c->host.resize(specs.size());
    for (size_t l = 0; l < specs.size(); ++l) build_level(P, specs[l], c->host[l]);
    std::vector<VankaFactors> VF(specs.size());
    std::vector<VankaDecoupled> VD(specs.size());
    std::vector<std::vector<double>> dense(specs.size());
    for (size_t l = 0; l + 1 < specs.size(); ++l) {
      const int form = vanka_form(*p, c->host[l]);
      if (form == STMG_VANKA_DECOUPLED || form == kFormDiagonal) {
        vanka_decoupled(c->host[l], VD[l], nthreads, form == kFormDiagonal);
        continue;
      }
      vanka_factors(c->host[l], VF[l], nthreads);
      if (form == STMG_VANKA_DENSE) vanka_dense(c->host[l], VF[l], dense[l], nthreads);
    }
    std::vector<double> cinv, cg;
    coarse_inverse(c->host.back(), cinv, cg);
    c->nd_coarse = c->host.back().ndofs;
    c->Cg = c->pool.upload<double>(cg, c->stream);
    c->Cinv = c->pool.upload<double>(cinv, c->stream);
    c->mom0 = c->pool.upload<double>(c->host[0].mom, c->stream);
    c->volume0 = c->host[0].volume;
    // the FP64 hierarchy always exists (operator, per-op calls); it holds the
    // smoother factors only in FP64 mode
    build_hier<double>(c, c->H64, VF, dense, VD, !c->mixed);
    if (c->mixed) build_hier<float>(c, c->H32, VF, dense, VD, true);
    int64_t ns = (int64_t)c->host[0].N * c->host[0].nt;
    c->partial = c->pool.alloc<double>((ns + 128) * 520 + 1024 * 128);
    c->dh = c->pool.alloc<double>(1024);
    c->w = c->pool.alloc<double>(c->host[0].ndofs);
    c->u = c->pool.alloc<double>(c->host[0].ndofs);
    c->dtmp = c->pool.alloc<double>(c->host[0].ndofs);
    if (c->mixed) c->zt = c->pool.alloc<double>(c->host[0].ndofs);
    // release host element matrices (kept: level sizes and tables)
    for (auto& L : c->host) {
      std::vector<double>().swap(L.Me);
      std::vector<double>().swap(L.Ae);
      std::vector<double>().swap(L.Be);
    }
  });
  if (rc != STMG_OK) {
    std::string m = c->err;
    c->pool.release();
    delete c;
    (void)m;
    return (stmg_status)rc;
  }
  *out = c;
  return STMG_OK;
}

stmg_status stmg_destroy(stmg_ctx* c) {
  if (!c) return STMG_EINVAL;
  (void)hipSetDevice(c->p.device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  c->pool.release();
  if (c->V) (void)hipFree(c->V);
  if (c->Z) (void)hipFree(c->Z);
  if (c->Z32) (void)hipFree(c->Z32);
  delete c;
  return STMG_OK;
}

const char* stmg_last_error(const stmg_ctx* c) { return c ? c->err.c_str() : "null context"; }

stmg_status stmg_sizes(const stmg_ctx* c, int level, int64_t* n_dofs, int64_t* nv, int64_t* np, int* n_levels) {
  if (!c || level < 0 || level >= (int)c->host.size()) return STMG_EINVAL;
  const LevelHost& L = c->host[level];
  if (n_dofs) *n_dofs = L.ndofs;
  if (nv) *nv = L.Mv;
  if (np) *np = L.Mp;
  if (n_levels) *n_levels = (int)c->host.size();
  return STMG_OK;
}

stmg_status stmg_set_phase_timing(stmg_ctx* c, int on) {
  if (!c) return STMG_EINVAL;
  c->phase_timing = on != 0;
  return STMG_OK;
}

stmg_status stmg_apply_operator(stmg_ctx* c, int level, const double* x, double* y) {
  if (!c || !x || !y || level < 0 || level >= (int)c->host.size()) return STMG_EINVAL;
  // the operator is always available in FP64 (the FGMRES operator)
  return (stmg_status)guarded(c, [&] {
    op_apply<double>(c, c->H64.L[level], x, x, y, 0);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_apply_operator_vcycle_precision(stmg_ctx* c, int level, const double* x, double* y) {
  if (!c || !x || !y || level < 0 || level >= (int)c->host.size()) return STMG_EINVAL;
  return (stmg_status)per_op(
      c, [&] { op_apply<double>(c, c->H64.L[level], x, x, y, 0); },
      [&] {
        DevLevel<float>& D = c->H32.L[level];
        HIPCHK(launch_cast_d2f(x, D.x, D.ndofs, c->stream));
        op_apply<float>(c, D, D.x, D.x, D.r, 0);
        HIPCHK(launch_cast_f2d(D.r, y, D.ndofs, c->stream));
      });
}

stmg_status stmg_set_option(stmg_ctx* c, int option, int64_t value) {
  if (!c || value < 0) return STMG_EINVAL;
  switch (option) {
    case STMG_OPT_APPLY_SUBINTERVALS:
      c->opt_apply_nper = (int)std::min<int64_t>(value, 1 << 20);
      return STMG_OK;
    case STMG_OPT_NET_CHUNK:
      c->opt_net_chunk = value;
      return STMG_OK;
    case STMG_OPT_INJECT_NONFINITE:
      c->opt_inject_nonfinite = value;
      return STMG_OK;
    case STMG_OPT_APPLY_LOOP_ORDER:
      if (value > 2) break;
      c->opt_apply_variant = (int)value;
      return STMG_OK;
    default:
      break;
  }
  c->err = "unknown option or value";
  return STMG_EINVAL;
}

stmg_status stmg_residual(stmg_ctx* c, int level, const double* b, const double* x, double* r) {
  if (!c || !b || !x || !r || level < 0 || level >= (int)c->host.size()) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    op_apply<double>(c, c->H64.L[level], x, b, r, 1);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_smooth(stmg_ctx* c, int level, const double* b, double* x, int steps) {
  if (!c || !b || !x || level < 0 || level + 1 >= (int)c->host.size() || steps < 0) return STMG_EINVAL;
  return (stmg_status)per_op(
      c, [&] { op_smooth<double>(c, c->H64.L[level], b, x, steps, false); },
      [&] {
        DevLevel<float>& D = c->H32.L[level];
        HIPCHK(launch_cast_d2f(b, D.b, D.ndofs, c->stream));
        HIPCHK(launch_cast_d2f(x, D.x, D.ndofs, c->stream));
        op_smooth<float>(c, D, D.b, D.x, steps, false);
        HIPCHK(launch_cast_f2d(D.x, x, D.ndofs, c->stream));
      });
}

stmg_status stmg_vanka_correction(stmg_ctx* c, int level, const double* r, double* x) {
  if (!c || !r || !x || level < 0 || level + 1 >= (int)c->host.size()) return STMG_EINVAL;
  return (stmg_status)per_op(
      c, [&] { op_vanka<double>(c, c->H64.L[level], r, x); },
      [&] {
        DevLevel<float>& D = c->H32.L[level];
        HIPCHK(launch_cast_d2f(r, D.r, D.ndofs, c->stream));
        HIPCHK(launch_cast_d2f(x, D.x, D.ndofs, c->stream));
        op_vanka<float>(c, D, D.r, D.x);
        HIPCHK(launch_cast_f2d(D.x, x, D.ndofs, c->stream));
      });
}

// ---------------------------------------------------------------------------
// Allocation-free Vanka correction.  Its scratch lives in one fixed device
// array per GPU (each device holds its own copy of this module variable).
// Host code never passes the array's name to a kernel or a copy: it uses the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[STMG_NOALLOC_SCRATCH_BYTES];

static unsigned char* scratch_address(int device) {
  static std::mutex m;
  static std::vector<unsigned char*> addr;
  std::lock_guard<std::mutex> g(m);
  if (device < 0) throw Error(STMG_EINVAL, "bad device ordinal");
  if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
  if (!addr[device]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));  // the current device's copy
    if (!p) throw DeviceError("hipGetSymbolAddress returned a null address");
    addr[device] = static_cast<unsigned char*>(p);
  }
  return addr[device];
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

stmg_status stmg_vanka_correction_noalloc(stmg_ctx* c, int level, const double* r, double* x) {
  if (!c || !r || !x || level < 0 || level + 1 >= (int)c->host.size()) return STMG_EINVAL;
  const LevelHost& L = c->host[level];
  const size_t elem = c->mixed ? sizeof(float) : sizeof(double);
  const size_t e_bytes = align256((size_t)L.ncells * L.d * L.nt * L.nloc * L.N * elem);
  const size_t v_bytes = c->mixed ? align256((size_t)L.ndofs * sizeof(float)) : 0;
  const size_t need = e_bytes + 2 * v_bytes;
  if (need > (size_t)STMG_NOALLOC_SCRATCH_BYTES)
    return (stmg_status)fail(c, STMG_EINVAL,
                             "level " + std::to_string(level) + " needs " + std::to_string(need) +
                                 " bytes of smoother scratch; the allocation-free correction holds " +
                                 std::to_string((size_t)STMG_NOALLOC_SCRATCH_BYTES));
  return (stmg_status)guarded(c, [&] {
    unsigned char* base = scratch_address(c->p.device);  // device is current (guarded)
    if (c->mixed) {
      DevLevel<float>& D = c->H32.L[level];
      float* E = reinterpret_cast<float*>(base);
      float* r32 = reinterpret_cast<float*>(base + e_bytes);
      float* x32 = reinterpret_cast<float*>(base + e_bytes + v_bytes);
      HIPCHK(launch_cast_d2f(r, r32, D.ndofs, c->stream));
      HIPCHK(launch_cast_d2f(x, x32, D.ndofs, c->stream));
      op_vanka_with<float>(c, D, r32, x32, E, false);
      HIPCHK(launch_cast_f2d(x32, x, D.ndofs, c->stream));
    } else {
      op_vanka_with<double>(c, c->H64.L[level], r, x, reinterpret_cast<double*>(base), false);
    }
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_kernel_time(stmg_ctx* c, int which, int level, int reps, double* avg_ms) {
  if (!c || !avg_ms || reps < 1 || level < 0 || level >= (int)c->host.size()) return STMG_EINVAL;
  if (which == 0 && level + 1 >= (int)c->host.size()) return STMG_EINVAL;
  if (which < 0 || which > 3) return STMG_EINVAL;
  if (which == 2 && (level + 1 >= (int)c->host.size() || vanka_form(c->p, c->host[level]) == STMG_VANKA_DENSE))
    return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    auto run = [&](auto& D) {
      using T = std::remove_reference_t<decltype(*D.x)>;
      HIPCHK(launch_fill<T>(D.b, T(1e-3), D.ndofs, c->stream));
      HIPCHK(launch_fill<T>(D.x, T(0), D.ndofs, c->stream));
      HIPCHK(launch_fill<T>(D.r, T(1e-3), D.ndofs, c->stream));
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, c->stream));
      for (int i = 0; i < reps; ++i) {
        if (which == 0) op_vanka<T>(c, D, D.r, D.x);
        else if (which == 1) op_apply<T>(c, D, D.x, D.b, D.r, 1);
        else if (which == 2 && (D.vform == STMG_VANKA_DECOUPLED || D.vform == kFormDiagonal))
          HIPCHK(launch_vanka_decoupled<T>(D.a, D.Asw, D.Bm, D.F, D.Hinv, D.coef, D.r, D.x, (T)c->p.omega, D.E,
                                           c->stream, false, false, D.vform == kFormDiagonal));
        else if (which == 2)
          HIPCHK(launch_vanka_factored<T>(D.a, D.Asw, D.Bm, D.F, D.Hinv, D.coef, D.r, D.x, (T)c->p.omega, D.E,
                                          c->stream, false));
        else
          HIPCHK(launch_apply<T>(D.a, D.geo, D.tab, D.x, D.b, D.r, 1, D.E, c->stream, false, c->opt_apply_nper,
                                 c->opt_apply_variant));
      }
      HIPCHK(hipEventRecord(e1, c->stream));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      *avg_ms = ms / reps;
    };
    if (c->mixed) run(c->H32.L[level]);
    else run(c->H64.L[level]);
  });
}

stmg_status stmg_restrict(stmg_ctx* c, int level, const double* fine, double* coarse) {
  if (!c || !fine || !coarse || level < 0 || level + 1 >= (int)c->host.size()) return STMG_EINVAL;
  return (stmg_status)per_op(
      c, [&] { op_restrict<double>(c, c->H64, level, fine, coarse); },
      [&] {
        DevLevel<float>& F = c->H32.L[level];
        DevLevel<float>& C = c->H32.L[level + 1];
        HIPCHK(launch_cast_d2f(fine, F.r, F.ndofs, c->stream));
        op_restrict<float>(c, c->H32, level, F.r, C.b);
        HIPCHK(launch_cast_f2d(C.b, coarse, C.ndofs, c->stream));
      });
}

stmg_status stmg_prolongate(stmg_ctx* c, int level, const double* coarse, double* fine) {
  if (!c || !fine || !coarse || level < 0 || level + 1 >= (int)c->host.size()) return STMG_EINVAL;
  return (stmg_status)per_op(
      c,
      [&] {
        HIPCHK(launch_fill<double>(fine, 0.0, c->host[level].ndofs, c->stream));
        op_prolongate_add<double>(c, c->H64, level, coarse, fine);
      },
      [&] {
        DevLevel<float>& F = c->H32.L[level];
        DevLevel<float>& C = c->H32.L[level + 1];
        HIPCHK(launch_cast_d2f(coarse, C.x, C.ndofs, c->stream));
        HIPCHK(launch_fill<float>(F.x, 0.0f, F.ndofs, c->stream));
        op_prolongate_add<float>(c, c->H32, level, C.x, F.x);
        HIPCHK(launch_cast_f2d(F.x, fine, F.ndofs, c->stream));
      });
}

stmg_status stmg_coarse_solve(stmg_ctx* c, const double* b, double* x) {
  if (!c || !b || !x) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    const LevelArgs& a = c->H64.L.back().a;
    HIPCHK(launch_coarse<double>(a.slab, a.Mv, a.nt, a.N, c->Cinv, c->Cg, b, x, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_vcycle(stmg_ctx* c, const double* b, double* x) {
  if (!c || !b || !x) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    precondition(c, b, x);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_project_pressure_mean_zero(stmg_ctx* c, double* x) {
  if (!c || !x) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    HIPCHK(launch_project_pressure(c->H64.L[0].a, c->mom0, c->volume0, x, c->partial, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_solve(stmg_ctx* c, const double* b, double* x, double rtol, int max_it, stmg_solve_info* info) {
  if (!c || !b || !x || !(rtol > 0) || max_it < 1) return STMG_EINVAL;
  int status = STMG_OK;
  int rc = guarded(c, [&] {
    const int64_t n = c->host[0].ndofs;
    // stride of the Krylov basis: a multiple of 4 KiB plus 2.25 KiB, so that
    // the vectors read side by side by the Gram-Schmidt passes start at
    // different offsets modulo large powers of two
    const int64_t ldv = (n + 511) / 512 * 512 + 288;
    hipStream_t s = c->stream;
    DevLevel<double>& L0 = c->H64.L[0];
    // Krylov basis capacity: bounded by max_it and by free device memory
    static_assert(STMG_RESTART <= kMaxFused, "restart length beyond the fused Gram-Schmidt kernels");
    int want = std::min(max_it, STMG_RESTART) + 1;
    if (c->cap < want) {
      size_t fr = 0, tot = 0;
      HIPCHK(hipMemGetInfo(&fr, &tot));
      int64_t fit = (int64_t)(0.45 * (double)fr / (2.0 * ldv * sizeof(double)));
      int cap = (int)std::max<int64_t>(8, std::min<int64_t>(want, fit));
      if (cap > c->cap) {
        if (c->V) (void)hipFree(c->V);
        if (c->Z) (void)hipFree(c->Z);
        if (c->Z32) (void)hipFree(c->Z32);
        c->V = nullptr;
        c->Z = nullptr;
        c->Z32 = nullptr;
        HIPCHK(hipMalloc(&c->V, (size_t)cap * ldv * sizeof(double)));
        if (c->mixed) HIPCHK(hipMalloc(&c->Z32, (size_t)cap * ldv * sizeof(float)));
        else HIPCHK(hipMalloc(&c->Z, (size_t)cap * ldv * sizeof(double)));
        c->cap = cap;
      }
    }
    const int m = c->cap - 1;
    c->history.clear();
    c->learned_disabled = false;
    c->learned_steps = 0;
    c->t_smooth.reset();
    c->t_vcyc.reset();
    c->t_op.reset();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    double bnorm = std::sqrt(dot(c, b, b, n));
    int total = 0, applications = 0, fallbacks = 0;
    double rel = 0.0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hv(m + 2), y(m);
    bool x_zero = true;
    while (true) {
      // explicit residual (b itself while x is still 0: b - S 0 = b exactly,
      // Dirichlet rows included)
      const double* r0 = b;
      double beta = bnorm;
      if (!x_zero) {
        if (c->phase_timing) c->t_op.a(s);
        op_apply<double>(c, L0, x, b, c->w, 1);
        if (c->phase_timing) c->t_op.b(s);
        beta = std::sqrt(dot(c, c->w, c->w, n));
        r0 = c->w;
      }
      rel = bnorm > 0 ? beta / bnorm : 0.0;
      c->history.push_back(rel);
      if (bnorm == 0.0 || beta <= rtol * bnorm || total >= max_it) {
        if (x_zero) HIPCHK(launch_fill<double>(x, 0.0, n, s));
        break;
      }
      // (mixed: the FP32 copy of V_0 is the first V-cycle's input)
      HIPCHK(launch_scale_copy(c->V, r0, 1.0 / beta, n, s, c->mixed ? c->H32.L[0].b : nullptr));
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int j = 0;
      // Arnoldi with classical Gram-Schmidt twice, lagged by one step: the
      // new direction u (after its first projection) is preconditioned as
      // it stands (FGMRES admits any z_j, and the V-cycle is homogeneous);
      // its second projection and normalisation are applied by the first
      // pass of the next step, which writes the final V_j.
      double* wv = c->w;
      double* uv = c->u;
      double invb = 0.0;
      while (j < m && total < max_it) {
        double* h1 = c->dh;
        double* h2n = c->dh + 256 + 128 * (j & 1);
        const double* h2p = c->dh + 256 + 128 * ((j + 1) & 1);
        std::vector<double> hh(j + 1), h2(j + 2);
        // z_j, w = S z_j and the Gram-Schmidt passes.  identity: z_j is the
        // V-cycle's input itself (the fallback step after a non-finite V-cycle;
        // FGMRES admits any z_j)
        auto arnoldi_step = [&](bool identity) {
          ++applications;
          if (c->mixed) {
            // z_j = V(v_j) in FP32 straight into the basis (its FP32 input was
            // written with v_j); w = S z_j in FP64 on its FP64 copy (an FP64
            // operator reading FP32 input directly runs slower)
            float* zj = c->Z32 + (size_t)j * ldv;
            if (identity) {
              // from the FP64 direction (the FP32 copy the V-cycle read was
              // overwritten by the failed step's second pass)
              HIPCHK(launch_cast_d2f(j == 0 ? c->V : uv, zj, n, s));
            } else {
              precondition_f32(c, zj);
              if (applications == c->opt_inject_nonfinite)
                HIPCHK(launch_fill<float>(zj, std::numeric_limits<float>::quiet_NaN(), n, s));
            }
            HIPCHK(launch_cast_f2d(zj, c->zt, n, s));
            if (c->phase_timing) c->t_op.a(s);
            op_apply<double>(c, L0, c->zt, c->zt, wv, 0);
            if (c->phase_timing) c->t_op.b(s);
          } else {
            double* zj = c->Z + (size_t)j * ldv;
            const double* vin = j == 0 ? c->V : uv;
            if (identity) {
              HIPCHK(hipMemcpyAsync(zj, vin, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            } else {
              precondition(c, vin, zj);
              if (applications == c->opt_inject_nonfinite)
                HIPCHK(launch_fill<double>(zj, std::numeric_limits<double>::quiet_NaN(), n, s));
            }
            if (c->phase_timing) c->t_op.a(s);
            op_apply<double>(c, L0, zj, zj, wv, 0);
            if (c->phase_timing) c->t_op.b(s);
          }
          // (mixed: pass 2 also writes the next direction in FP32, the next V-cycle's input)
          HIPCHK(launch_lcgs2(c->V, ldv, j, j > 0 ? 1 : 0, uv, h2p, invb, wv, n, c->partial, h1, h2n,
                              c->mixed ? c->H32.L[0].b : nullptr, s));
          HIPCHK(hipMemcpyAsync(hh.data(), h1, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
          HIPCHK(hipMemcpyAsync(h2.data(), h2n, h2.size() * sizeof(double), hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
          bool finite = true;
          for (double v : hh) finite = finite && std::isfinite(v);
          for (double v : h2) finite = finite && std::isfinite(v);
          return finite;
        };
        if (!arnoldi_step(false)) {
          // a non-finite preconditioned direction (e.g. an FP32 overflow in
          // the V-cycle): redo this step with the unpreconditioned direction.
          // Pass 1 rewrites V_j from the same pending vector, so nothing
          // else needs undoing.
          ++fallbacks;
          if (!arnoldi_step(true)) throw Error(STMG_ESINGULAR, "FGMRES direction is not finite");
        }
        std::fill(hv.begin(), hv.end(), 0.0);
        double q2 = 0.0;
        for (int i = 0; i <= j; ++i) {
          hv[i] = hh[i] + h2[i];
          q2 += h2[i] * h2[i];
        }
        // |w - V h2| from |w|^2 - |h2|^2 (h2 is a rounding-level correction)
        const double hn = std::sqrt(std::max(0.0, h2[j + 1] - q2));
        hv[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
          double t = cs[i] * hv[i] + sn[i] * hv[i + 1];
          hv[i + 1] = -sn[i] * hv[i] + cs[i] * hv[i + 1];
          hv[i] = t;
        }
        double den = std::hypot(hv[j], hv[j + 1]);
        cs[j] = hv[j] / den;
        sn[j] = hv[j + 1] / den;
        hv[j] = den;
        hv[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        for (int i = 0; i <= j + 1; ++i) H[(size_t)i * m + j] = hv[i];
        ++total;
        ++j;
        c->history.push_back(std::fabs(g[j]) / bnorm);
        if (!std::isfinite(g[j])) throw Error(STMG_ESINGULAR, "FGMRES produced a non-finite residual");
        if (std::fabs(g[j]) <= rtol * bnorm || hn == 0.0) break;
        invb = 1.0 / hn;
        std::swap(wv, uv);  // the projected w becomes the pending direction
      }
      for (int i = j - 1; i >= 0; --i) {
        double t = g[i];
        for (int k2 = i + 1; k2 < j; ++k2) t -= H[(size_t)i * m + k2] * y[k2];
        y[i] = t / H[(size_t)i * m + i];
      }
      HIPCHK(hipMemcpyAsync(c->dh, y.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
      // (x = 0 before the first combination: it is written, not read)
      if (c->mixed) HIPCHK(launch_combine_f32(x, c->Z32, ldv, j, c->dh, n, s, x_zero));
      else HIPCHK(launch_combine(x, c->Z, ldv, j, c->dh, n, s, x_zero));
      x_zero = false;
    }
    HIPCHK(launch_project_pressure(L0.a, c->mom0, c->volume0, x, c->partial, s));
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->iterations = total;
      info->rel_residual = rel;
      info->t_solve_s = ms * 1e-3;
      if (c->phase_timing) {
        info->t_smoother_s = c->t_smooth.total_s();
        double tv = c->t_vcyc.total_s();
        info->t_mg_other_s = tv - info->t_smoother_s;
        info->t_operator_s = c->t_op.total_s();
        info->t_other_s = info->t_solve_s - tv - info->t_operator_s;
      }
      info->learned_disabled = c->learned_disabled ? 1 : 0;
      info->vcycle_fallbacks = fallbacks;
      info->learned_steps = c->learned_steps;
      info->history_len = (int)c->history.size();
      info->history = c->history.data();
    }
    if (!(rel <= rtol)) status = STMG_ENOCONV;
  });
  if (rc != STMG_OK) return (stmg_status)rc;
  if (status != STMG_OK) c->err = "FGMRES did not reach the tolerance within max_it";
  return (stmg_status)status;
}

// ------------------------------------------------------------ time marching
stmg_status stmg_time_nodes(const stmg_ctx* c, double* t_hat) {
  if (!c || !t_hat) return STMG_EINVAL;
  const LevelHost& L = c->host[0];
  for (int a = 0; a < L.nt; ++a) t_hat[a] = L.td.t[a];
  return STMG_OK;
}

// b = f - S_full gD - C^1 v0 on free rows, 0 on Dirichlet rows, where gD
// holds g's Dirichlet velocity entries and zeros elsewhere (f, g, v0 may be null)
static void slab_rhs_impl(stmg_ctx* c, const double* f, const double* v0, const double* g, double* b) {
  DevLevel<double>& D = c->H64.L[0];
  const int64_t n = D.ndofs;
  if (!c->slab_b) {
    c->slab_b = c->pool.alloc<double>(n);
    c->slab_g = c->pool.alloc<double>(n);
  }
  HIPCHK(launch_fill<double>(c->slab_g, 0.0, n, c->stream));
  if (g) HIPCHK(launch_set_dirichlet(D.a, g, c->slab_g, c->stream));
  const double* fz = f;
  if (!fz) {  // zero forcing
    HIPCHK(launch_fill<double>(b, 0.0, n, c->stream));
    fz = b;
  }
  HIPCHK(launch_slab_rhs(D.a, D.geo, D.tab, fz, c->slab_g, v0, b, D.E, c->stream));
}

stmg_status stmg_slab_rhs(stmg_ctx* c, const double* f, const double* v0, const double* g, double* b) {
  if (!c || !b) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    slab_rhs_impl(c, f, v0, g, b);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_slab_end_value(stmg_ctx* c, const double* x, double* v_end) {
  if (!c || !x || !v_end) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    const LevelHost& L = c->host[0];
    const double* src = x + (int64_t)(L.N - 1) * L.slab + (int64_t)(L.nt - 1) * L.Mv;
    HIPCHK(hipMemcpyAsync(v_end, src, (size_t)L.Mv * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_solve_slab(stmg_ctx* c, const double* f, const double* v0, const double* g, double* x, double rtol,
                            int max_it, stmg_solve_info* info) {
  if (!c || !x || !(rtol > 0) || max_it < 1) return STMG_EINVAL;
  int rc = guarded(c, [&] {
    const int64_t n = c->host[0].ndofs;
    if (!c->slab_b) {
      c->slab_b = c->pool.alloc<double>(n);
      c->slab_g = c->pool.alloc<double>(n);
    }
    slab_rhs_impl(c, f, v0, g, c->slab_b);
  });
  if (rc != STMG_OK) return (stmg_status)rc;
  // the homogeneous system for x - gD, then the Dirichlet values
  const stmg_status st = stmg_solve(c, c->slab_b, x, rtol, max_it, info);
  if (st != STMG_OK && st != STMG_ENOCONV) return st;
  if (g) {
    rc = guarded(c, [&] {
      HIPCHK(launch_set_dirichlet(c->H64.L[0].a, g, x, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    });
    if (rc != STMG_OK) return (stmg_status)rc;
  }
  return st;
}

stmg_status stmg_march(stmg_ctx* c, int n_slabs, const double* f, const double* g, const double* v0, double* x,
                       double rtol, int max_it, int* iterations) {
  if (!c || !x || n_slabs < 1 || !(rtol > 0) || max_it < 1) return STMG_EINVAL;
  const LevelHost& L = c->host[0];
  const int64_t n = L.ndofs;
  for (int s = 0; s < n_slabs; ++s) {
    // the previous slab's end value: the last temporal dof (the Radau point
    // at the right end) of its last subinterval
    const double* vin = s == 0 ? v0 : x + (s - 1) * n + (int64_t)(L.N - 1) * L.slab + (int64_t)(L.nt - 1) * L.Mv;
    stmg_solve_info info;
    const stmg_status st = stmg_solve_slab(c, f ? f + s * n : nullptr, vin, g ? g + s * n : nullptr, x + s * n,
                                           rtol, max_it, &info);
    if (iterations) iterations[s] = info.iterations;
    if (st != STMG_OK) {
      if (st == STMG_ENOCONV) c->err = "slab " + std::to_string(s) + ": FGMRES did not reach the tolerance";
      return st;
    }
  }
  return STMG_OK;
}

stmg_status stmg_learned_load(stmg_ctx* c, const float* w, size_t n) {
  if (!c || !w || n != (size_t)kNetParams) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    net_alloc(c, 4096);
    HIPCHK(hipMemcpyAsync(c->net.w, w, kNetParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(launch_fill<float>(c->net.m, 0.0f, kNetParams, c->stream));
    HIPCHK(launch_fill<float>(c->net.v, 0.0f, kNetParams, c->stream));
    HIPCHK(net_pack(c->net, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_learned_weights(const stmg_ctx* cc, float* w, size_t n) {
  stmg_ctx* c = const_cast<stmg_ctx*>(cc);
  if (!c || !w || n != (size_t)kNetParams || !c->net_ready) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    HIPCHK(hipMemcpyAsync(w, c->net.w, kNetParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

// learned work vectors (two per level reached by the correction), in the V-cycle's precision
static void lsave_alloc(stmg_ctx* c) {
  if (!c->lsave.empty()) return;
  for (size_t l = 0; l < c->host.size(); ++l) {
    size_t bytes = (c->mixed ? sizeof(float) : sizeof(double));
    bool use = net_route(c, (int)l) != 0;
    c->lsave.push_back(use ? c->pool.alloc<char>(c->host[l].ndofs * bytes) : nullptr);
    c->lsave.push_back(use ? c->pool.alloc<char>(c->host[l].ndofs * bytes) : nullptr);
  }
}

stmg_status stmg_learned_enable(stmg_ctx* c, int on) {
  if (!c || on < 0 || on > 2) return STMG_EINVAL;
  if (on && !c->net_ready) {
    c->err = "load weights before enabling the learned correction";
    return STMG_EINVAL;
  }
  return (stmg_status)guarded(c, [&] {
    if (on) lsave_alloc(c);
    c->learned_on = on != 0;
    if (on) c->learned_reading = on;
  });
}

stmg_status stmg_learned_record(stmg_ctx* c, const double* b, const double* xstar, double* r_out, double* e_out) {
  if (!c || !b || !xstar || !r_out || !e_out || c->host.size() < 2) return STMG_EINVAL;
  if (c->mixed) { c->err = "record pairs with an FP64 context"; return STMG_EINVAL; }
  if (!net_level(c->H64.L[0].a)) { c->err = "pairs need a 3D Q2/P1 x DG(1) finest level"; return STMG_EINVAL; }
  return (stmg_status)guarded(c, [&] {
    Hier<double>& H = c->H64;
    DevLevel<double>& D = H.L[0];
    const int64_t n = D.ndofs;
    HIPCHK(hipMemcpyAsync(D.b, b, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(launch_fill<double>(D.x, 0.0, n, c->stream));
    auto record = [&](int k) {
      op_apply<double>(c, D, D.x, D.b, r_out + k * n, 1);
      HIPCHK(hipMemcpyAsync(e_out + k * n, xstar, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(launch_axpy<double>(e_out + k * n, -1.0, D.x, n, c->stream));
    };
    op_smooth<double>(c, D, D.b, D.x, c->p.nu_pre, true);
    record(0);
    op_apply<double>(c, D, D.x, D.b, D.r, 1);
    op_restrict<double>(c, H, 0, D.r, H.L[1].b);
    vcycle<double>(c, H, 1);
    op_prolongate_add<double>(c, H, 0, H.L[1].x, D.x);
    op_smooth<double>(c, D, D.b, D.x, c->p.nu_post, false);
    record(1);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

// Adam over device FP32 pairs (the body of stmg_learned_train_pairs)
static void train_pairs_impl(stmg_ctx* c, const float* rp, const float* ep, int n_pairs, uint64_t seed, int epochs,
                             int batch, float lr, float* loss_hist) {
  const LevelArgs& a = c->H64.L[0].a;
  {
    net_alloc(c, batch);
    if (batch > c->net.cap) throw Error(STMG_EINVAL, "batch too large");
    const int64_t nd = c->host[0].ndofs;
    const int64_t per = (int64_t)a.N * (a.Mp / a.C);
    const int64_t nchunk = (per + batch - 1) / batch;
    std::vector<int64_t> order((size_t)n_pairs * nchunk);
    uint64_t st = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto rnd = [&]() {  // 64-bit LCG, top bits
      st = st * 6364136223846793005ULL + 1442695040888963407ULL;
      return st >> 11;
    };
    int t = 0;
    size_t h = 0;
    for (int ep_i = 0; ep_i < epochs; ++ep_i) {
      for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
      for (size_t i = order.size(); i > 1; --i) std::swap(order[i - 1], order[rnd() % i]);
      for (int64_t job : order) {
        const int64_t pair = job / nchunk, first = (job % nchunk) * batch;
        const int64_t cnt = std::min<int64_t>(batch, per - first);
        HIPCHK(net_inputs<float>(a, c->net, rp + pair * nd, ep + pair * nd, first, cnt, c->stream));
        HIPCHK(net_forward(c->net, cnt, c->stream, true));
        HIPCHK(net_loss(c->net, cnt, c->stream));
        HIPCHK(net_backward(c->net, cnt, c->stream));
        HIPCHK(net_adam(c->net, ++t, lr, c->stream));
        double red[2];
        HIPCHK(hipMemcpyAsync(red, c->net.red, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (loss_hist) loss_hist[h++] = red[1] > 0 ? (float)(red[0] / red[1]) : 0.0f;
      }
    }
  }
}

stmg_status stmg_learned_train_pairs(stmg_ctx* c, const float* rp, const float* ep, int n_pairs, uint64_t seed,
                                     int epochs, int batch, float lr, float* loss_hist) {
  if (!c || !rp || !ep || n_pairs < 1 || epochs < 1 || batch < 8 || !(lr > 0) || !c->net_ready)
    return STMG_EINVAL;
  if (!net_level(c->H64.L[0].a)) { c->err = "training needs a 3D Q2/P1 x DG(1) finest level"; return STMG_EINVAL; }
  return (stmg_status)guarded(c, [&] { train_pairs_impl(c, rp, ep, n_pairs, seed, epochs, batch, lr, loss_hist); });
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): one 64-bit output per
// counter step; uniform doubles from its top 53 bits.
namespace {
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }  // [0, 1)
};
}  // namespace

stmg_status stmg_learned_train(stmg_ctx* c, int n_pairs, uint64_t seed, int epochs, float lr, float* weights_out) {
  if (!c || n_pairs < 2 || epochs < 1 || !(lr > 0) || !weights_out || c->host.size() < 2) return STMG_EINVAL;
  if (c->mixed) { c->err = "train in an FP64 context"; return STMG_EINVAL; }
  if (!net_level(c->H64.L[0].a)) { c->err = "training needs a 3D Q2/P1 x DG(1) finest level"; return STMG_EINVAL; }
  const LevelHost& L = c->host[0];
  const int64_t nd = L.ndofs;
  const int n_forc = (n_pairs + 1) / 2, np = 2 * n_forc;
  constexpr int kBatch = 4096;
  double *b = nullptr, *xs = nullptr, *r2 = nullptr, *e2 = nullptr;
  float *rp = nullptr, *ep = nullptr;
  auto release = [&] {
    for (void* p : {(void*)b, (void*)xs, (void*)r2, (void*)e2, (void*)rp, (void*)ep})
      if (p) (void)hipFree(p);
  };
  int rc = guarded(c, [&] {
    if (!c->net_ready) {  // He-normal initialisation drawn from the seed (Box-Muller)
      SplitMix64 g{seed ^ 0x5DEECE66DULL};
      std::vector<float> w0(kNetParams);
      const int cin[3] = {15, 32, 32}, cout[3] = {32, 32, 14};
      size_t o = 0;
      for (int l = 0; l < 3; ++l) {
        const double sd = std::sqrt(2.0 / (cin[l] * 27.0));
        for (int i = 0; i < cout[l] * cin[l] * 27; ++i) {
          const double u1 = 1.0 - g.uniform(), u2 = g.uniform();
          w0[o++] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2));
        }
      }
      net_alloc(c, kBatch);
      HIPCHK(hipMemcpyAsync(c->net.w, w0.data(), kNetParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
      HIPCHK(launch_fill<float>(c->net.m, 0.0f, kNetParams, c->stream));
      HIPCHK(launch_fill<float>(c->net.v, 0.0f, kNetParams, c->stream));
      HIPCHK(net_pack(c->net, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    }
    HIPCHK(hipMalloc(&b, nd * sizeof(double)));
    HIPCHK(hipMalloc(&xs, nd * sizeof(double)));
    HIPCHK(hipMalloc(&r2, 2 * nd * sizeof(double)));
    HIPCHK(hipMalloc(&e2, 2 * nd * sizeof(double)));
    HIPCHK(hipMalloc(&rp, (size_t)np * nd * sizeof(float)));
    HIPCHK(hipMalloc(&ep, (size_t)np * nd * sizeof(float)));
  });
  if (rc != STMG_OK) { release(); return (stmg_status)rc; }
  // forcings: velocity entries U[-1, 1) on interior nodes, zero Dirichlet
  // entries and pressure rows (a consistent right-hand side, Eq. (DefB))
  std::vector<double> bh(nd);
  for (int f = 0; f < n_forc && rc == STMG_OK; ++f) {
    SplitMix64 g{seed * 0x9E3779B97F4A7C15ULL + (uint64_t)f + 1};
    std::fill(bh.begin(), bh.end(), 0.0);
    for (int n = 0; n < L.N; ++n)
      for (int a = 0; a < L.nt; ++a)
        for (int comp = 0; comp < L.d; ++comp)
          for (int64_t node = 0; node < L.nodes; ++node) {
            const int64_t gx = node % L.nn, gy = (node / L.nn) % L.nn, gz = node / ((int64_t)L.nn * L.nn);
            const bool bnd = gx == 0 || gx == L.nn - 1 || gy == 0 || gy == L.nn - 1 ||
                             (L.d == 3 && (gz == 0 || gz == L.nn - 1));
            const double u = 2.0 * g.uniform() - 1.0;
            if (!bnd) bh[(size_t)(n * L.slab + a * L.Mv + comp * L.nodes + node)] = u;
          }
    rc = guarded(c, [&] {
      HIPCHK(hipMemcpyAsync(b, bh.data(), nd * sizeof(double), hipMemcpyHostToDevice, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    });
    if (rc != STMG_OK) break;
    const bool was_on = c->learned_on;
    c->learned_on = false;  // the reference solution and the pairs come from plain multigrid
    stmg_solve_info info;
    rc = stmg_solve(c, b, xs, 1e-12, 200, &info);
    if (rc == STMG_OK) rc = stmg_learned_record(c, b, xs, r2, e2);
    c->learned_on = was_on;
    if (rc != STMG_OK) break;
    rc = guarded(c, [&] {
      HIPCHK(launch_cast_d2f(r2, rp + (size_t)2 * f * nd, 2 * nd, c->stream));
      HIPCHK(launch_cast_d2f(e2, ep + (size_t)2 * f * nd, 2 * nd, c->stream));
    });
  }
  if (rc == STMG_OK)
    rc = guarded(c, [&] {
      train_pairs_impl(c, rp, ep, np, seed, epochs, kBatch, lr, nullptr);
      HIPCHK(hipMemcpyAsync(weights_out, c->net.w, kNetParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    });
  (void)hipStreamSynchronize(c->stream);
  release();
  return (stmg_status)rc;
}

stmg_status stmg_learned_correction(stmg_ctx* c, int level, const double* r, double* u) {
  if (!c || !r || !u || level < 0 || level >= (int)c->host.size() || !c->net_ready) return STMG_EINVAL;
  const int route = net_route(c, level);
  if (route == 0) return STMG_EINVAL;
  if (route == 2 && c->mixed) {
    c->err = "the correction through the next level is evaluated in an FP64 context";
    return STMG_EINVAL;
  }
  return (stmg_status)guarded(c, [&] {
    if (route == 2) lsave_alloc(c);
    learned_correction_at<double>(c, level, route, r, u);
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

stmg_status stmg_learned_gradient(stmg_ctx* c, int level, const double* r, const double* e, float* grad, double* loss) {
  if (!c || !r || !e || !grad || level < 0 || level >= (int)c->host.size() || !c->net_ready) return STMG_EINVAL;
  const LevelArgs& a = c->H64.L[level].a;
  if (!net_level(a)) return STMG_EINVAL;
  const int64_t total = (int64_t)a.N * (a.Mp / a.C);
  if (total > c->net.cap) return STMG_EINVAL;
  return (stmg_status)guarded(c, [&] {
    net_alloc(c, total);
    HIPCHK(net_inputs<double>(a, c->net, r, e, 0, total, c->stream));
    HIPCHK(net_forward(c->net, total, c->stream, true));
    HIPCHK(net_loss(c->net, total, c->stream));
    HIPCHK(net_backward(c->net, total, c->stream));
    std::vector<float> g(kNetParams);
    double red[2];
    HIPCHK(hipMemcpyAsync(g.data(), c->net.g, kNetParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(red, c->net.red, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < kNetParams; ++i) grad[i] = (float)(g[i] / red[1]);
    if (loss) *loss = red[0] / red[1];
  });
}

}  // extern "C"
