// Device kernels of the hp space-time multigrid for gfx950 (wave64).
//
// Data layout (Eq. (DefX)): X = (V_1, P_1, ..., V_N, P_N), V_n^a component-major
// over the global Gauss-Lobatto nodes, P_n^a cell-major over Legendre modes.
// Scatter-adds to velocity nodes shared by cells are made race-free and
// deterministic by 2^d-colouring the cells (cells of one colour share no node).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace stmg {

namespace {

__device__ __forceinline__ int64_t vidx(const LevelArgs& L, int n, int a, int comp, int64_t g) {
  return (int64_t)n * L.slab + (int64_t)a * L.Mv + (int64_t)comp * L.nodes + g;
}
__device__ __forceinline__ int64_t pidx(const LevelArgs& L, int n, int a, int64_t cell, int l) {
  return (int64_t)n * L.slab + (int64_t)L.nt * L.Mv + (int64_t)a * L.Mp + cell * L.C + l;
}

// Number of cells of one colour and the coordinates of its w-th cell.
__device__ __forceinline__ int64_t color_count(int n, int d, int color) {
  int64_t t = 1;
  for (int j = 0; j < d; ++j) t *= (n - ((color >> j) & 1) + 1) / 2;
  return t;
}
__device__ __forceinline__ void color_cell(int n, int d, int color, int64_t w, int* cc) {
  for (int j = 0; j < 3; ++j) cc[j] = 0;
  for (int j = 0; j < d; ++j) {
    int bit = (color >> j) & 1;
    int cnt = (n - bit + 1) / 2;
    cc[j] = 2 * (int)(w % cnt) + bit;
    w /= cnt;
  }
}

// Global node of local node i (Q per direction) in cell cc; Dirichlet flag
// and valence (number of cells sharing the node).
template <int D>
__device__ __forceinline__ int64_t gnode(const LevelArgs& L, const int* cc, int i, bool& free_, int& val) {
  int64_t g = 0, st = 1;
  free_ = true;
  val = 1;
  for (int j = 0; j < D; ++j) {
    int ij = i % L.Q;
    i /= L.Q;
    int gj = cc[j] * L.q + ij;
    if (gj == 0 || gj == L.nn - 1) free_ = false;
    else if (gj % L.q == 0) val *= 2;
    g += gj * st;
    st *= L.nn;
  }
  return g;
}

// One 1D contraction along `dir` through LDS: out(p) = sum_t M[pd][t] buf(p|pd=t)
// (trans: M[t][pd]).
template <typename T, int Q>
__device__ __forceinline__ T contract(const T* buf, int p, int dir, const T* M, bool trans) {
  const int stride = dir == 0 ? 1 : (dir == 1 ? Q : Q * Q);
  const int pd = (p / stride) % Q;
  const T* b = buf + (p - pd * stride);
  T s = 0;
#pragma unroll
  for (int t = 0; t < Q; ++t) s += (trans ? M[t * Q + pd] : M[pd * Q + t]) * b[t * stride];
  return s;
}

}  // namespace

// =====================================================================
// Space-time operator.  One work item = (cell of one colour, subinterval n);
// one thread per quadrature point (Q^d <= 64), 64 / Q^d cells per wave.
// For every temporal dof a of subinterval n:
//   y_v += K_ab M x_v[n,b] + c_a A_nu x_v[n,a] - c_a B^T x_p[n,a] - phi_a(-1) M x_v[n-1,k]
//   y_p += -c_a B x_v[n,a]
// with c_a = (tau/2) w_a (Eq. (InAlg), (DefDtauh), (GloSys); M^tau diagonal).
// =====================================================================
template <typename T, int D, int Q>
__global__ __launch_bounds__(64) void k_apply(LevelArgs L, const double* __restrict__ verts,
                                              const T* __restrict__ nu_q, T nu_const, const T* __restrict__ tab,
                                              const T* __restrict__ x, const T* __restrict__ b,
                                              T* __restrict__ y, T* __restrict__ E, int mode) {
  constexpr int NL = D == 2 ? Q * Q : Q * Q * Q;
  constexpr int CPB = 64 / NL;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int nt = L.nt, C = L.C;
  const int tabn = 2 * Q * Q + 2 * Q + nt * nt + 2 * nt + NL * C;
  for (int t = threadIdx.x; t < tabn; t += blockDim.x) smem[t] = tab[t];
  const T* sS = smem;
  const T* sDg = sS + Q * Q;
  const T* sgx = sDg + Q * Q;
  const T* sgw = sgx + Q;
  const T* sK = sgw + Q;
  const T* sphi = sK + nt * nt;
  const T* scoef = sphi + nt;
  const T* spsi = scoef + nt;
  const int per_cell = 5 * NL + nt * C;
  T* cbase = smem + ((tabn + 1) & ~1);

  const int tid = threadIdx.x;
  int slot = tid / NL;
  const int p = tid % NL;
  const int64_t total = L.Mp / L.C;
  const int64_t w = (int64_t)blockIdx.x * CPB + slot;
  bool active = slot < CPB && w < total;
  const T sgn = mode ? T(-1) : T(1);
  if (slot > CPB) slot = CPB;
  T* bufA = cbase + slot * per_cell;
  T* bufB = bufA + NL;
  T* g0 = bufB + NL;
  T* g1 = g0 + NL;
  T* g2 = g1 + NL;
  T* pv = g2 + NL;
  const int n = blockIdx.y;

  const int64_t cell = active ? w : 0;
  int cc[3] = {(int)(cell % L.n), (int)((cell / L.n) % L.n), D == 3 ? (int)(cell / ((int64_t)L.n * L.n)) : 0};
  bool fr;
  int val;
  const int64_t g = gnode<D>(L, cc, p, fr, val);
  const int pq[3] = {p % Q, (p / Q) % Q, p / (Q * Q)};
  __syncthreads();

  // ---- geometry at this quadrature point: J of the multilinear map
  T J[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) J[i][j] = 0;
  T xi[D];
#pragma unroll
  for (int j = 0; j < D; ++j) xi[j] = sgx[pq[j]];
#pragma unroll
  for (int v = 0; v < (1 << D); ++v) {
    int64_t vi = 0, st = 1;
    T f[D], df[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      int bit = (v >> j) & 1;
      vi += (cc[j] + bit) * st;
      st *= (L.n + 1);
      f[j] = bit ? xi[j] : T(1) - xi[j];
      df[j] = bit ? T(1) : T(-1);
    }
#pragma unroll
    for (int gdir = 0; gdir < D; ++gdir) {
      T dN = 1;
#pragma unroll
      for (int j = 0; j < D; ++j) dN *= (j == gdir) ? df[j] : f[j];
#pragma unroll
      for (int i = 0; i < D; ++i) J[i][gdir] += (T)verts[vi * D + i] * dN;
    }
  }
  T Ji[D][D], det;
  if constexpr (D == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    T id = T(1) / det;
    Ji[0][0] = J[1][1] * id; Ji[0][1] = -J[0][1] * id; Ji[1][0] = -J[1][0] * id; Ji[1][1] = J[0][0] * id;
  } else {
    T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    T id = T(1) / det;
    Ji[0][0] = c00 * id; Ji[1][0] = c01 * id; Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  }
  T jxw = det;
#pragma unroll
  for (int j = 0; j < D; ++j) jxw *= sgw[pq[j]];
  const T nu = nu_q ? nu_q[cell * NL + p] : nu_const;

  // ---- values at the quadrature points of all temporal dofs (and of the
  // last dof of the previous subinterval)
  int cur = 0;
  auto pp_interp = [&](T v) -> T {
#pragma unroll
    for (int dir = 0; dir < D; ++dir) {
      T* buf = cur ? bufB : bufA;
      buf[p] = v;
      __syncthreads();
      v = contract<T, Q>(buf, p, dir, sS, false);
      cur ^= 1;
    }
    return v;
  };
  T ub[4][D];
  T up[D];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int comp = 0; comp < D; ++comp) {
      ub[b][comp] = 0;
      if (b < nt) {
        T v = (active && fr) ? x[vidx(L, n, b, comp, g)] : T(0);
        ub[b][comp] = pp_interp(v);
      }
    }
#pragma unroll
  for (int comp = 0; comp < D; ++comp) {
    T v = (active && fr && n > 0) ? x[vidx(L, n - 1, nt - 1, comp, g)] : T(0);
    up[comp] = (n > 0) ? pp_interp(v) : T(0);
  }
  for (int t = p; t < nt * C; t += NL) pv[t] = active ? x[pidx(L, n, t / C, cell, t % C)] : T(0);
  __syncthreads();

#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (a >= nt) break;
    const T ca = scoef[a];
    T pres = 0;
    for (int l = 0; l < C; ++l) pres += spsi[p * C + l] * pv[a * C + l];
    T div = 0;
#pragma unroll
    for (int comp = 0; comp < D; ++comp) {
      T W = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b < nt) W += sK[a * nt + b] * ub[b][comp];
      W -= sphi[a] * up[comp];
      // reference gradient of u_a at the Gauss points (collocation derivative)
      T gr[D];
      {
        T* buf = cur ? bufB : bufA;
        buf[p] = ub[a][comp];
        __syncthreads();
#pragma unroll
        for (int dir = 0; dir < D; ++dir) gr[dir] = contract<T, Q>(buf, p, dir, sDg, false);
        cur ^= 1;
      }
      // physical gradient J^{-T} gr, flux F = c_a (nu grad u - p e_comp), G = J^{-1} F JxW
      T gp[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        T s = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) s += Ji[j][i] * gr[j];
        gp[i] = s;
      }
      div += gp[comp];
      T Fl[D];
#pragma unroll
      for (int i = 0; i < D; ++i) Fl[i] = ca * nu * gp[i] - (i == comp ? ca * pres : T(0));
      T Gr[D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T s = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) s += Ji[j][i] * Fl[i];
        Gr[j] = s * jxw;
      }
      g0[p] = Gr[0];
      g1[p] = Gr[1];
      if constexpr (D == 3) g2[p] = Gr[2];
      __syncthreads();
      T Z = W * jxw + contract<T, Q>(g0, p, 0, sDg, true) + contract<T, Q>(g1, p, 1, sDg, true);
      if constexpr (D == 3) Z += contract<T, Q>(g2, p, 2, sDg, true);
      // back to the nodes: transposed interpolation
#pragma unroll
      for (int dir = 0; dir < D; ++dir) {
        T* buf = cur ? bufB : bufA;
        buf[p] = Z;
        __syncthreads();
        Z = contract<T, Q>(buf, p, dir, sS, true);
        cur ^= 1;
      }
      if (active)
        E[cell * (int64_t)D * nt * NL * L.N + ((int64_t)(n * nt + a) * D + comp) * NL + p] = Z;
    }
    // continuity: y_p[l] += -c_a sum_q psi_l div JxW
    g0[p] = -ca * div * jxw;
    __syncthreads();
    if (active && p < C) {
      T s = 0;
      for (int q = 0; q < NL; ++q) s += spsi[q * C + p] * g0[q];
      const int64_t id = pidx(L, n, a, cell, p);
      y[id] = (mode ? b[id] : T(0)) + sgn * s;
    }
  }
}

// Velocity rows of y = S x (mode 0) / y = b - S x (mode 1): sum the cell
// contributions of every node in a fixed order; Dirichlet rows are the identity.
template <typename T, int D>
__global__ void k_apply_gather(LevelArgs L, const T* __restrict__ E, const T* __restrict__ x,
                               const T* __restrict__ b, T* __restrict__ y, int mode) {
  const int64_t per = (int64_t)L.nt * D * L.nodes;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)L.N * per) return;
  const int n = (int)(idx / per);
  int64_t rem = idx % per;
  const int a = (int)(rem / ((int64_t)D * L.nodes));
  rem %= (int64_t)D * L.nodes;
  const int comp = (int)(rem / L.nodes);
  const int64_t g = rem % L.nodes;
  const int64_t id = vidx(L, n, a, comp, g);
  int gj[3] = {(int)(g % L.nn), (int)((g / L.nn) % L.nn), D == 3 ? (int)(g / ((int64_t)L.nn * L.nn)) : 0};
  int cj[3][2], ij[3][2], nj[3] = {1, 1, 1};
  bool bnd = false;
  for (int j = 0; j < D; ++j) {
    if (gj[j] == 0 || gj[j] == L.nn - 1) bnd = true;
    int c = gj[j] / L.q, i = gj[j] % L.q;
    if (c == L.n) { c = L.n - 1; i = L.q; }
    if (i == 0 && c > 0) {
      cj[j][0] = c - 1; ij[j][0] = L.q;
      cj[j][1] = c;     ij[j][1] = 0;
      nj[j] = 2;
    } else {
      cj[j][0] = c; ij[j][0] = i;
    }
  }
  if (bnd) {
    y[id] = mode ? b[id] - x[id] : x[id];
    return;
  }
  const int64_t stride = (int64_t)D * L.nt * L.nloc * L.N;
  const int64_t off = ((int64_t)(n * L.nt + a) * D + comp) * L.nloc;
  T s = 0;
  for (int u = 0; u < (D == 3 ? nj[2] : 1); ++u)
    for (int v = 0; v < nj[1]; ++v)
      for (int w = 0; w < nj[0]; ++w) {
        int64_t cell = cj[0][w] + (int64_t)L.n * (cj[1][v] + (int64_t)L.n * (D == 3 ? cj[2][u] : 0));
        int i = ij[0][w] + L.Q * (ij[1][v] + L.Q * (D == 3 ? ij[2][u] : 0));
        s += E[cell * stride + off + i];
      }
  y[id] = mode ? b[id] - s : s;
}

template <typename T, int D, int Q>
static hipError_t apply_impl(const LevelArgs& L, const double* verts, const T* nu_q, T nu_const, const T* tab,
                             const T* x, const T* b, T* y, int mode, T* E, hipStream_t s) {
  constexpr int NL = D == 2 ? Q * Q : Q * Q * Q;
  constexpr int CPB = 64 / NL;
  const int tabn = table_size(Q, L.nt, NL, L.C);
  size_t shm = sizeof(T) * (((tabn + 1) & ~1) + (CPB + 1) * (5 * NL + L.nt * L.C));
  int64_t ncells = L.Mp / L.C;
  dim3 grid((unsigned)((ncells + CPB - 1) / CPB), (unsigned)L.N);
  k_apply<T, D, Q><<<grid, 64, shm, s>>>(L, verts, nu_q, nu_const, tab, x, b, y, E, mode);
  int64_t nv = (int64_t)L.N * L.nt * D * L.nodes;
  k_apply_gather<T, D><<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(L, E, x, b, y, mode);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply(const LevelArgs& L, const double* verts, const T* nu_q, T nu_const, const T* tab,
                        const T* x, const T* b, T* y, int mode, T* E, hipStream_t s) {
  if (L.d == 2 && L.Q == 3) return apply_impl<T, 2, 3>(L, verts, nu_q, nu_const, tab, x, b, y, mode, E, s);
  if (L.d == 2 && L.Q == 4) return apply_impl<T, 2, 4>(L, verts, nu_q, nu_const, tab, x, b, y, mode, E, s);
  if (L.d == 3 && L.Q == 3) return apply_impl<T, 3, 3>(L, verts, nu_q, nu_const, tab, x, b, y, mode, E, s);
  if (L.d == 3 && L.Q == 4) return apply_impl<T, 3, 4>(L, verts, nu_q, nu_const, tab, x, b, y, mode, E, s);
  return hipErrorInvalidValue;
}

// =====================================================================
// Cell Vanka, Schur-factored local inverse (Eq. (vanka0), (vanka)).
// One work group per spatial cell, all N subintervals at once (the local
// matrix is the same for every subinterval).  Local velocity rows (a, i) per
// component; pressure rows q = (a, l).
//   Z = A_s^{-1} R               (MFMA: mp x mp times mp x (d N), one pass over A_s^{-1})
//   y_p = H^{-1} (D Z - r_p),    y_c = z_c - F_c y_p
//   x_p += omega y_p             (pressure dofs belong to one cell)
//   E   = y_v                    (velocity: summed per node by k_vanka_gather)
// MFMA 16x16x4 operand order: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element v holds D[row][l%16] with row = 4 (l/16) + v for FP32
// and row = l/16 + 4 v for FP64 (both checked on gfx950).
// =====================================================================
template <typename T>
struct mfma_vec;
template <>
struct mfma_vec<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane / 16) + v; }
};
template <>
struct mfma_vec<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return lane / 16 + 4 * v; }
};

template <typename T, int D, int N>
__global__ __launch_bounds__(256) void k_vanka_mfma(LevelArgs L, const T* __restrict__ Asw,
                                                    const T* __restrict__ Bm, const T* __restrict__ F,
                                                    const T* __restrict__ Hinv, const T* __restrict__ coef,
                                                    const T* __restrict__ r, T* __restrict__ x, T omega,
                                                    T* __restrict__ E) {
  constexpr int DN = D * N;
  constexpr int NCT = (DN + 15) / 16;  // column tiles of 16
  constexpr int DNP = NCT * 16;
  typedef typename mfma_vec<T>::v4 v4;
  const int nl = L.nloc, nt = L.nt, C = L.C, m = nt * nl, P = nt * C;
  const int mp = (m + 15) & ~15, nkb = mp / 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* RZ = reinterpret_cast<T*>(smem_raw);  // R (B-operand order), then Z (row-major mp x DNP)
  T* Rp = RZ + (size_t)mp * DNP;
  T* S = Rp + P * N;
  T* YP = S + P * N;
  T* sc = YP + P * N;
  const int64_t cell = blockIdx.x;
  int cc[3] = {(int)(cell % L.n), (int)((cell / L.n) % L.n), (int)(cell / ((int64_t)L.n * L.n))};
  const int tid = threadIdx.x;
  // ---- gather r into B-operand order; padded rows/columns are zero
  for (int t = tid; t < mp * DNP; t += blockDim.x) RZ[t] = 0;
  __syncthreads();
  for (int t = tid; t < m * DN; t += blockDim.x) {
    int i = t % nl, rest = t / nl;
    int a = rest % nt;
    rest /= nt;
    int comp = rest % D, n = rest / D;
    bool fr;
    int val;
    int64_t g = gnode<D>(L, cc, i, fr, val);
    int K = a * nl + i, col = comp * N + n;
    int ct = col / 16, jj = col % 16, kb = K / 16, rem = K % 16;
    RZ[(((size_t)ct * nkb + kb) * 64 + jj + 16 * (rem / 4)) * 4 + (rem % 4)] = fr ? r[vidx(L, n, a, comp, g)] : T(0);
  }
  for (int t = tid; t < P * N; t += blockDim.x) {
    int q = t % P, n = t / P;
    Rp[q * N + n] = r[pidx(L, n, q / C, cell, q % C)];
  }
  if (tid < nt) sc[tid] = coef[tid];
  __syncthreads();
  // ---- Z = A_s^{-1} R on the matrix cores
  const int wave = tid / 64, lane = tid % 64;
  const int nwave = blockDim.x / 64;
  const T* A = Asw + (size_t)cell * mp * mp;
  v4 acc[4][NCT];  // up to 4 row tiles per wave (mp <= 256)
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int t = wave + it * nwave;
    if (t < nkb) {
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[it][ct] = v4{0, 0, 0, 0};
      const T* At = A + (size_t)t * nkb * 256;
      for (int kb = 0; kb < nkb; ++kb) {
        const T* ap = At + ((size_t)kb * 64 + lane) * 4;
        T a0 = ap[0], a1 = ap[1], a2 = ap[2], a3 = ap[3];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const T* bp = RZ + (((size_t)ct * nkb + kb) * 64 + lane) * 4;
          acc[it][ct] = mfma_vec<T>::mma(a0, bp[0], acc[it][ct]);
          acc[it][ct] = mfma_vec<T>::mma(a1, bp[1], acc[it][ct]);
          acc[it][ct] = mfma_vec<T>::mma(a2, bp[2], acc[it][ct]);
          acc[it][ct] = mfma_vec<T>::mma(a3, bp[3], acc[it][ct]);
        }
      }
    }
  }
  __syncthreads();  // every wave is done reading R
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int t = wave + it * nwave;
    if (t < nkb)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          RZ[(size_t)(t * 16 + mfma_vec<T>::row(lane, v)) * DNP + ct * 16 + lane % 16] = acc[it][ct][v];
  }
  __syncthreads();
  T* Z = RZ;
  // ---- pressure Schur complement
  const T* B = Bm + cell * (int64_t)C * D * nl;
  for (int t = tid; t < P * N; t += blockDim.x) {
    int q = t / N, n = t % N, a = q / C, l = q % C;
    T s = 0;
    for (int comp = 0; comp < D; ++comp)
      for (int i = 0; i < nl; ++i) s += B[(l * D + comp) * nl + i] * Z[(size_t)(a * nl + i) * DNP + comp * N + n];
    S[q * N + n] = -sc[a] * s - Rp[q * N + n];
  }
  __syncthreads();
  const T* H = Hinv + cell * (int64_t)P * P;
  for (int t = tid; t < P * N; t += blockDim.x) {
    int pp = t / N, n = t % N;
    T s = 0;
    for (int q = 0; q < P; ++q) s += H[q * P + pp] * S[q * N + n];
    YP[pp * N + n] = s;
    x[pidx(L, n, pp / C, cell, pp % C)] += omega * s;
  }
  __syncthreads();
  // ---- velocity: y = z - F y_p into the cell-local buffer, layout
  // E[cell][(n nt + a) D + comp][i]
  const T* Fc = F + cell * (int64_t)D * m * P;
  T* Ec = E + cell * (int64_t)D * m * N;
  for (int row2 = tid; row2 < D * m; row2 += blockDim.x) {
    int comp = row2 / m, row = row2 % m, a = row / nl, i = row % nl;
    T acc2[N];
#pragma unroll
    for (int n = 0; n < N; ++n) acc2[n] = Z[(size_t)row * DNP + comp * N + n];
    for (int q = 0; q < P; ++q) {
      T f = Fc[((int64_t)comp * P + q) * m + row];
#pragma unroll
      for (int n = 0; n < N; ++n) acc2[n] -= f * YP[q * N + n];
    }
#pragma unroll
    for (int n = 0; n < N; ++n) Ec[((int64_t)(n * nt + a) * D + comp) * nl + i] = acc2[n];
  }
}

// x_v += omega / valence * (sum over the cells containing the node of E),
// cells taken in a fixed order (deterministic); Dirichlet nodes unchanged.
template <typename T, int D>
__global__ void k_vanka_gather(LevelArgs L, const T* __restrict__ E, T* __restrict__ x, T omega) {
  const int64_t per = (int64_t)L.nt * D * L.nodes;  // velocity dofs of one subinterval
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)L.N * per) return;
  const int n = (int)(idx / per);
  int64_t rem = idx % per;
  const int a = (int)(rem / ((int64_t)D * L.nodes));
  rem %= (int64_t)D * L.nodes;
  const int comp = (int)(rem / L.nodes);
  const int64_t g = rem % L.nodes;
  int gj[3] = {(int)(g % L.nn), (int)((g / L.nn) % L.nn), D == 3 ? (int)(g / ((int64_t)L.nn * L.nn)) : 0};
  // cells containing the node along each direction: (cell, local index)
  int cj[3][2], ij[3][2], nj[3];
  for (int j = 0; j < D; ++j) {
    if (gj[j] == 0 || gj[j] == L.nn - 1) return;  // Dirichlet
    int c = gj[j] / L.q, i = gj[j] % L.q;
    if (i == 0) {
      cj[j][0] = c - 1; ij[j][0] = L.q;
      cj[j][1] = c;     ij[j][1] = 0;
      nj[j] = 2;
    } else {
      cj[j][0] = c; ij[j][0] = i;
      nj[j] = 1;
    }
  }
  const int64_t stride = (int64_t)D * L.nt * L.nloc * L.N;  // per cell
  const int64_t off = ((int64_t)(n * L.nt + a) * D + comp) * L.nloc;
  T s = 0;
  int val = 1;
  for (int j = 0; j < D; ++j) val *= nj[j];
  for (int u = 0; u < (D == 3 ? nj[2] : 1); ++u)
    for (int v = 0; v < nj[1]; ++v)
      for (int w = 0; w < nj[0]; ++w) {
        int64_t cell = cj[0][w] + (int64_t)L.n * (cj[1][v] + (int64_t)L.n * (D == 3 ? cj[2][u] : 0));
        int i = ij[0][w] + L.Q * (ij[1][v] + L.Q * (D == 3 ? ij[2][u] : 0));
        s += E[cell * stride + off + i];
      }
  x[vidx(L, n, a, comp, g)] += omega / T(val) * s;
}

template <typename T, int D, int N>
static hipError_t vanka_fact_impl(const LevelArgs& L, const T* Asw, const T* Bm, const T* F, const T* Hinv,
                                  const T* coef, const T* r, T* x, T omega, T* E, hipStream_t s) {
  const int m = L.nt * L.nloc, P = L.nt * L.C, mp = (m + 15) & ~15;
  constexpr int DNP = ((D * N + 15) / 16) * 16;
  if (mp / 16 > 16) return hipErrorInvalidValue;  // at most 4 row tiles per wave
  size_t shm = sizeof(T) * ((size_t)mp * DNP + 3 * (size_t)P * N + L.nt + 2);
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  int64_t ncells = L.Mp / L.C;
  k_vanka_mfma<T, D, N><<<(unsigned)ncells, 256, shm, s>>>(L, Asw, Bm, F, Hinv, coef, r, x, omega, E);
  int64_t nv = (int64_t)L.N * L.nt * D * L.nodes;
  k_vanka_gather<T, D><<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(L, E, x, omega);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vanka_gather_only(const LevelArgs& L, const T* E, T* x, T omega, hipStream_t s) {
  int64_t nv = (int64_t)L.N * L.nt * L.d * L.nodes;
  if (L.d == 3) k_vanka_gather<T, 3><<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(L, E, x, omega);
  else k_vanka_gather<T, 2><<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(L, E, x, omega);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vanka_factored(const LevelArgs& L, const T* Asw, const T* Bm, const T* F, const T* Hinv,
                                 const T* coef, const T* r, T* x, T omega, T* E, hipStream_t s) {
#define STMG_VF(DD, NN) \
  if (L.d == DD && L.N == NN) return vanka_fact_impl<T, DD, NN>(L, Asw, Bm, F, Hinv, coef, r, x, omega, E, s);
  STMG_VF(2, 1) STMG_VF(2, 2) STMG_VF(2, 4) STMG_VF(2, 8)
  STMG_VF(3, 1) STMG_VF(3, 2) STMG_VF(3, 4) STMG_VF(3, 8)
#undef STMG_VF
  return hipErrorInvalidValue;
}

// Dense local inverse: Y (b x N) = A^{-1} (b x b, column-major) R (b x N);
// local order: velocity (comp, a, i), then pressure (a, l).
template <typename T, int D, int N>
__global__ __launch_bounds__(256) void k_vanka_dense(LevelArgs L, int color, const T* __restrict__ Ainv,
                                                     const T* __restrict__ r, T* __restrict__ x, T omega) {
  const int nl = L.nloc, nt = L.nt, C = L.C, m = nt * nl, P = nt * C, bs = D * m + P;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* R = reinterpret_cast<T*>(smem_raw);
  int cc[3];
  color_cell(L.n, D, color, blockIdx.x, cc);
  const int64_t cell = cc[0] + (int64_t)L.n * (cc[1] + (int64_t)L.n * cc[2]);
  const int tid = threadIdx.x;
  for (int t = tid; t < bs * N; t += blockDim.x) {
    int row = t % bs, n = t / bs;
    T v;
    if (row < D * m) {
      int comp = row / m, a = (row % m) / nl, i = row % nl;
      bool fr;
      int val;
      int64_t g = gnode<D>(L, cc, i, fr, val);
      v = fr ? r[vidx(L, n, a, comp, g)] : T(0);
    } else {
      int q = row - D * m;
      v = r[pidx(L, n, q / C, cell, q % C)];
    }
    R[row * N + n] = v;
  }
  __syncthreads();
  const T* A = Ainv + cell * (int64_t)bs * bs;
  for (int row = tid; row < bs; row += blockDim.x) {
    T acc[N];
#pragma unroll
    for (int n = 0; n < N; ++n) acc[n] = 0;
    int j = 0;
    for (; j + 4 <= bs; j += 4) {
      T a0 = A[(int64_t)j * bs + row], a1 = A[(int64_t)(j + 1) * bs + row];
      T a2 = A[(int64_t)(j + 2) * bs + row], a3 = A[(int64_t)(j + 3) * bs + row];
#pragma unroll
      for (int n = 0; n < N; ++n)
        acc[n] += a0 * R[j * N + n] + a1 * R[(j + 1) * N + n] + a2 * R[(j + 2) * N + n] + a3 * R[(j + 3) * N + n];
    }
    for (; j < bs; ++j) {
      T a0 = A[(int64_t)j * bs + row];
#pragma unroll
      for (int n = 0; n < N; ++n) acc[n] += a0 * R[j * N + n];
    }
    if (row < D * m) {
      int comp = row / m, a = (row % m) / nl, i = row % nl;
      bool fr;
      int val;
      int64_t g = gnode<D>(L, cc, i, fr, val);
      if (fr) {
        T wgt = omega / T(val);
#pragma unroll
        for (int n = 0; n < N; ++n) x[vidx(L, n, a, comp, g)] += wgt * acc[n];
      }
    } else {
      int q = row - D * m;
#pragma unroll
      for (int n = 0; n < N; ++n) x[pidx(L, n, q / C, cell, q % C)] += omega * acc[n];
    }
  }
}

template <typename T, int D, int N>
static hipError_t vanka_dense_impl(const LevelArgs& L, const T* Ainv, const T* r, T* x, T omega, hipStream_t s) {
  const int bs = D * L.nt * L.nloc + L.nt * L.C;
  size_t shm = sizeof(T) * (size_t)bs * N;
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  for (int color = 0; color < (1 << D); ++color) {
    int64_t tot = 1;
    for (int j = 0; j < D; ++j) tot *= (L.n - ((color >> j) & 1) + 1) / 2;
    if (tot == 0) continue;
    k_vanka_dense<T, D, N><<<(unsigned)tot, 256, shm, s>>>(L, color, Ainv, r, x, omega);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vanka_dense(const LevelArgs& L, const T* Ainv, const T* r, T* x, T omega, hipStream_t s) {
#define STMG_VD(DD, NN) \
  if (L.d == DD && L.N == NN) return vanka_dense_impl<T, DD, NN>(L, Ainv, r, x, omega, s);
  STMG_VD(2, 1) STMG_VD(2, 2) STMG_VD(2, 4) STMG_VD(2, 8)
  STMG_VD(3, 1) STMG_VD(3, 2) STMG_VD(3, 4) STMG_VD(3, 8)
#undef STMG_VD
  return hipErrorInvalidValue;
}

// =====================================================================
// Transfers (App. A).  Velocity: the global embedding is a tensor product of
// 1D matrices (reference-coordinate interpolation on a structured mesh), so
// it is applied as d batched 1D passes.  Pressure: per-cell embedding of the
// parent's Legendre expansion.  Time: a small dense matrix over slices.
// =====================================================================
struct ArrLayout {  // where array b of a batch of d-dimensional node arrays lives
  int level;        // 1: level vector (n, a, comp) blocks; 0: compact
  int nt, D;
  int64_t slab, Mv, nodes, compact_stride;
};
__device__ __forceinline__ int64_t arr_base(const ArrLayout& A, int64_t b) {
  if (!A.level) return b * A.compact_stride;
  int comp = (int)(b % A.D);
  int64_t t = b / A.D;
  int a = (int)(t % A.nt);
  int64_t n = t / A.nt;
  return n * A.slab + (int64_t)a * A.Mv + (int64_t)comp * A.nodes;
}

// out[b][..o..] (+)= sum_t M[o][t] in[b][..t..] along `axis`;
// dims_out[3] (x, y, z), nin = extent of the input along the axis.
template <typename T>
__global__ void k_vpass(const T* __restrict__ in, ArrLayout li, T* __restrict__ out, ArrLayout lo, int64_t nb,
                        int d, int axis, int dx, int dy, int dz, int nin, const T* __restrict__ M,
                        const int* __restrict__ lo_, const int* __restrict__ hi_, int mask_in, int mask_out,
                        int accumulate) {
  const int64_t per = (int64_t)dx * dy * dz;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * per) return;
  int64_t b = idx / per, e = idx % per;
  int o[3] = {(int)(e % dx), (int)((e / dx) % dy), (int)(e / ((int64_t)dx * dy))};
  int dims_out[3] = {dx, dy, dz};
  int dims_in[3] = {dx, dy, dz};
  dims_in[axis] = nin;
  const T* src = in + arr_base(li, b);
  int64_t strides[3] = {1, dims_in[0], (int64_t)dims_in[0] * dims_in[1]};
  int64_t base = 0;
  for (int j = 0; j < d; ++j)
    if (j != axis) base += o[j] * strides[j];
  bool in_bnd_other = false;
  if (mask_in)
    for (int j = 0; j < d; ++j)
      if (j != axis && (o[j] == 0 || o[j] == dims_in[j] - 1)) in_bnd_other = true;
  const int oa = o[axis];
  T s = 0;
  if (!in_bnd_other) {
    for (int t = lo_[oa]; t < hi_[oa]; ++t) {
      if (mask_in && (t == 0 || t == nin - 1)) continue;
      s += M[(int64_t)oa * nin + t] * src[base + t * strides[axis]];
    }
  }
  if (mask_out)
    for (int j = 0; j < d; ++j)
      if (o[j] == 0 || o[j] == dims_out[j] - 1) s = 0;
  T* dst = out + arr_base(lo, b) + e;
  if (accumulate) *dst += s;
  else *dst = s;
}

// Pressure: prolong (dir 0): xf[cf][l] += sum_m E[pos][l][m] xc[parent][m];
// restrict (dir 1): bc[cp][m] = sum_children sum_l E[pos][l][m] rf[child][l].
template <typename T>
__global__ void k_ppass(const T* __restrict__ in, T* __restrict__ out, int nslices, int nt_in, int nt_out,
                        int64_t slab_in, int64_t off_in, int64_t Mp_in, int64_t slab_out, int64_t off_out,
                        int64_t Mp_out, int d, int n_out, int n_in, int C_out, int C_in, const T* __restrict__ E,
                        int npos, int dir, int Cf, int Cc) {
  int64_t ncell = 1;
  for (int j = 0; j < d; ++j) ncell *= n_out;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nslices * ncell * C_out) return;
  int l = (int)(idx % C_out);
  int64_t c = (idx / C_out) % ncell;
  int s = (int)(idx / (C_out * ncell));
  int n = s / nt_out, a = s % nt_out;
  int cc[3] = {(int)(c % n_out), (int)((c / n_out) % n_out), (int)(c / ((int64_t)n_out * n_out))};
  const T* src = in + (int64_t)n * slab_in + off_in + (int64_t)a * Mp_in;
  T* dst = out + (int64_t)n * slab_out + off_out + (int64_t)a * Mp_out;
  T v = 0;
  if (dir == 0) {
    int ratio = n_out / n_in;
    int pos = 0;
    int64_t par = 0, st = 1;
    for (int j = 0; j < d; ++j) {
      if (ratio == 2) pos |= (cc[j] & 1) << j;
      par += (cc[j] / ratio) * st;
      st *= n_in;
    }
    const T* e = E + ((int64_t)pos * Cf + l) * Cc;
    for (int mm = 0; mm < C_in; ++mm) v += e[mm] * src[par * C_in + mm];
    dst[c * C_out + l] += v;
  } else {
    int ratio = n_in / n_out;
    for (int pos = 0; pos < npos; ++pos) {
      int64_t ch = 0, st = 1;
      for (int j = 0; j < d; ++j) {
        int o = ratio == 2 ? (pos >> j) & 1 : 0;
        ch += (cc[j] * ratio + o) * st;
        st *= n_in;
      }
      for (int lf = 0; lf < C_in; ++lf) v += E[((int64_t)pos * Cf + lf) * Cc + l] * src[ch * C_in + lf];
    }
    dst[c * C_out + l] = v;
  }
}

// Time: out slice so (+)= sum_si M[so][si] in slice si, for velocity and pressure blocks.
template <typename T>
__global__ void k_tpass(const T* __restrict__ in, T* __restrict__ out, int ns_in, int nt_in, int ns_out, int nt_out,
                        int64_t Mv, int64_t Mp, const T* __restrict__ M, int trans, int accumulate) {
  const int64_t per = Mv + Mp;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ns_out * per) return;
  int so = (int)(idx / per);
  int64_t j = idx % per;
  const int64_t slab_in = (int64_t)nt_in * per, slab_out = (int64_t)nt_out * per;
  auto off = [&](int s, int nt, int64_t slab) -> int64_t {
    int n = s / nt, a = s % nt;
    return j < Mv ? n * slab + (int64_t)a * Mv + j : n * slab + (int64_t)nt * Mv + (int64_t)a * Mp + (j - Mv);
  };
  T v = 0;
  for (int si = 0; si < ns_in; ++si) {
    T w = trans ? M[(int64_t)si * ns_out + so] : M[(int64_t)so * ns_in + si];
    if (w != T(0)) v += w * in[off(si, nt_in, slab_in)];
  }
  T* d = out + off(so, nt_out, slab_out);
  if (accumulate) *d += v;
  else *d = v;
}

static inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
static void space_velocity(const LevelArgs& Li, const LevelArgs& Lo, int nt, int N, const T* M, const int* lo,
                           const int* hi, const T* in, ArrLayout li, T* out, ArrLayout lout, T* tmp1, T* tmp2,
                           bool restrict_, hipStream_t s) {
  // Li: spatial sizes of the input, Lo: of the output
  const int d = Li.d;
  const int64_t nb = (int64_t)N * nt * d;
  int dims[3] = {Li.nn, Li.nn, d == 3 ? Li.nn : 1};
  const T* src = in;
  ArrLayout ls = li;
  for (int axis = 0; axis < d; ++axis) {
    int nin = dims[axis];
    dims[axis] = Lo.nn;
    bool last = axis == d - 1;
    T* dst = last ? out : (axis == 0 ? tmp1 : tmp2);
    ArrLayout ld = lout;
    if (!last) {
      ld.level = 0;
      ld.compact_stride = (int64_t)dims[0] * dims[1] * dims[2];
    }
    int64_t tot = nb * dims[0] * dims[1] * dims[2];
    k_vpass<T><<<nblk(tot), 256, 0, s>>>(src, ls, dst, ld, nb, d, axis, dims[0], dims[1], dims[2], nin, M, lo, hi,
                                         axis == 0 ? 1 : 0, (last && restrict_) ? 1 : 0, (last && !restrict_) ? 1 : 0);
    src = dst;
    ls = ld;
  }
}

template <typename T>
hipError_t launch_prolongate_add(const LevelArgs& F, const LevelArgs& Cs, const TransferDev& t, const T* P1,
                                 const int* rlo, const int* rhi, const T* E, const T* Pt, const T* xc, T* xf,
                                 T* tmp1, T* tmp2, T* tmp3, hipStream_t s) {
  // time first (on the coarse spatial grid): tmp3 = Pt xc, layout (N_f, nt_f, coarse space)
  const T* src = xc;
  int64_t slab_src = Cs.slab;
  int nt_src = Cs.nt;
  if (t.time_change) {
    int64_t tot = (int64_t)t.ntf * (Cs.Mv + Cs.Mp);
    k_tpass<T><<<nblk(tot), 256, 0, s>>>(xc, tmp3, t.ntc, Cs.nt, t.ntf, F.nt, Cs.Mv, Cs.Mp, Pt, 0, 0);
    src = tmp3;
    slab_src = (int64_t)F.nt * (Cs.Mv + Cs.Mp);
    nt_src = F.nt;
  }
  ArrLayout li{1, nt_src, F.d, slab_src, Cs.Mv, Cs.nodes, 0};
  ArrLayout lo{1, F.nt, F.d, F.slab, F.Mv, F.nodes, 0};
  space_velocity<T>(Cs, F, F.nt, F.N, P1, rlo, rhi, src, li, xf, lo, tmp1, tmp2, false, s);
  int64_t tot = (int64_t)F.N * F.nt * (int64_t)(F.Mp);
  k_ppass<T><<<nblk(tot), 256, 0, s>>>(src, xf, F.N * F.nt, nt_src, F.nt, slab_src, (int64_t)nt_src * Cs.Mv, Cs.Mp,
                                       F.slab, (int64_t)F.nt * F.Mv, F.Mp, F.d, F.n, Cs.n, F.C, Cs.C, E, t.npos, 0,
                                       F.C, Cs.C);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const LevelArgs& F, const LevelArgs& Cs, const TransferDev& t, const T* P1T,
                           const int* clo, const int* chi, const T* E, const T* Pt, const T* rf, T* bc, T* tmp1,
                           T* tmp2, T* tmp3, hipStream_t s) {
  T* dst = t.time_change ? tmp3 : bc;
  int64_t slab_dst = t.time_change ? (int64_t)F.nt * (Cs.Mv + Cs.Mp) : Cs.slab;
  ArrLayout li{1, F.nt, F.d, F.slab, F.Mv, F.nodes, 0};
  ArrLayout lo{1, F.nt, F.d, slab_dst, Cs.Mv, Cs.nodes, 0};
  space_velocity<T>(F, Cs, F.nt, F.N, P1T, clo, chi, rf, li, dst, lo, tmp1, tmp2, true, s);
  int64_t ncc = 1;
  for (int j = 0; j < F.d; ++j) ncc *= Cs.n;
  int64_t tot = (int64_t)F.N * F.nt * ncc * Cs.C;
  k_ppass<T><<<nblk(tot), 256, 0, s>>>(rf, dst, F.N * F.nt, F.nt, F.nt, F.slab, (int64_t)F.nt * F.Mv, F.Mp, slab_dst,
                                       (int64_t)F.nt * Cs.Mv, Cs.Mp, F.d, Cs.n, F.n, Cs.C, F.C, E, t.npos, 1, F.C,
                                       Cs.C);
  if (t.time_change) {
    int64_t tot2 = (int64_t)t.ntc * (Cs.Mv + Cs.Mp);
    k_tpass<T><<<nblk(tot2), 256, 0, s>>>(tmp3, bc, t.ntf, F.nt, t.ntc, Cs.nt, Cs.Mv, Cs.Mp, Pt, 1, 0);
  }
  return hipGetLastError();
}

// =====================================================================
// Coarse solve: the coarsest slab matrix is block lower-bidiagonal in time,
// so x_n = Dinv b_n - G x_{n-1,last} (one launch per subinterval, one wave
// per row, FP64 arithmetic).
// =====================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_coarse(int64_t slab, int64_t Mv, int nt, int n,
                                                const double* __restrict__ Di, const double* __restrict__ G,
                                                const T* __restrict__ b, T* __restrict__ x) {
  int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  int lane = threadIdx.x % 64;
  double s = 0.0;
  if (row < slab) {
    const T* bn = b + (int64_t)n * slab;
    for (int64_t j = lane; j < slab; j += 64) s += Di[row * slab + j] * (double)bn[j];
    if (n > 0) {
      const T* xp = x + (int64_t)(n - 1) * slab + (int64_t)(nt - 1) * Mv;
      for (int64_t j = lane; j < Mv; j += 64) s -= G[row * Mv + j] * (double)xp[j];
    }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (row < slab && lane == 0) x[(int64_t)n * slab + row] = (T)s;
}

template <typename T>
hipError_t launch_coarse(int64_t slab, int64_t Mv, int nt, int N, const double* Dinv, const double* G, const T* b,
                         T* x, hipStream_t s) {
  for (int n = 0; n < N; ++n) k_coarse<T><<<(unsigned)((slab + 3) / 4), 256, 0, s>>>(slab, Mv, nt, n, Dinv, G, b, x);
  return hipGetLastError();
}

// =====================================================================
// Vector kernels (deterministic reductions: fixed-order two-pass sums).
// =====================================================================
template <typename T>
__global__ void k_fill(T* x, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
template <typename T>
__global__ void k_axpy(T* y, T a, const T* x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}
__global__ void k_d2f(const double* a, float* b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void k_f2d(const float* a, double* b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

template <typename T>
hipError_t launch_fill(T* x, T v, int64_t n, hipStream_t s) {
  if (n > 0) k_fill<T><<<nblk(n), 256, 0, s>>>(x, v, n);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_axpy(T* y, T a, const T* x, int64_t n, hipStream_t s) {
  if (n > 0) k_axpy<T><<<nblk(n), 256, 0, s>>>(y, a, x, n);
  return hipGetLastError();
}
hipError_t launch_cast_d2f(const double* a, float* b, int64_t n, hipStream_t s) {
  k_d2f<<<nblk(n), 256, 0, s>>>(a, b, n);
  return hipGetLastError();
}
hipError_t launch_cast_f2d(const float* a, double* b, int64_t n, hipStream_t s) {
  k_f2d<<<nblk(n), 256, 0, s>>>(a, b, n);
  return hipGetLastError();
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x / 64); ++i) s += sh[i];
  return s;
}

constexpr int kDotBlocks = 512;

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ V, int64_t ldv,
                                                     const double* __restrict__ w, int64_t n,
                                                     double* __restrict__ partial) {
  __shared__ double sh[4];
  const int vi = blockIdx.y;
  const double* v = V + (int64_t)vi * ldv;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += v[i] * w[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[(int64_t)vi * kDotBlocks + blockIdx.x] = s;
}
__global__ void k_dot_final(const double* __restrict__ partial, int nv, double* __restrict__ out) {
  int vi = blockIdx.x * blockDim.x + threadIdx.x;
  if (vi >= nv) return;
  double s = 0.0;
  for (int b = 0; b < kDotBlocks; ++b) s += partial[(int64_t)vi * kDotBlocks + b];
  out[vi] = s;
}

hipError_t launch_multidot(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* partial,
                           double* out, hipStream_t s) {
  k_dot_partial<<<dim3(kDotBlocks, nv), 256, 0, s>>>(V, ldv, w, n, partial);
  k_dot_final<<<(nv + 63) / 64, 64, 0, s>>>(partial, nv, out);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot_t(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                               double* __restrict__ partial) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)a[i] * (double)b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
template <typename T>
hipError_t launch_dot(const T* a, const T* b, int64_t n, double* partial, double* out, hipStream_t s) {
  k_dot_t<T><<<kDotBlocks, 256, 0, s>>>(a, b, n, partial);
  k_dot_final<<<1, 64, 0, s>>>(partial, 1, out);
  return hipGetLastError();
}
template hipError_t launch_dot<double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template hipError_t launch_dot<float>(const float*, const float*, int64_t, double*, double*, hipStream_t);

__global__ void k_multi_axpy(double* __restrict__ w, const double* __restrict__ V, int64_t ldv, int nv,
                             const double* __restrict__ h, int64_t n, double sign) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nv; ++k) s += h[k] * V[(int64_t)k * ldv + i];
  w[i] += sign * s;
}
hipError_t launch_multi_axpy(double* w, const double* V, int64_t ldv, int nv, const double* h, int64_t n,
                             hipStream_t s) {
  k_multi_axpy<<<nblk(n), 256, 0, s>>>(w, V, ldv, nv, h, n, -1.0);
  return hipGetLastError();
}
hipError_t launch_combine(double* x, const double* Z, int64_t ldz, int nv, const double* y, int64_t n,
                          hipStream_t s) {
  k_multi_axpy<<<nblk(n), 256, 0, s>>>(x, Z, ldz, nv, y, n, 1.0);
  return hipGetLastError();
}
__global__ void k_scale_copy(double* y, const double* x, double inv, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] * inv;
}
hipError_t launch_scale_copy(double* y, const double* x, double inv, int64_t n, hipStream_t s) {
  k_scale_copy<<<nblk(n), 256, 0, s>>>(y, x, inv, n);
  return hipGetLastError();
}

// pressure mean per slice: partial sums over cells, then subtract from mode 0
__global__ __launch_bounds__(256) void k_pmean_partial(LevelArgs L, const double* __restrict__ mom,
                                                       const double* __restrict__ x, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int sl = blockIdx.y, n = sl / L.nt, a = sl % L.nt;
  const double* p = x + (int64_t)n * L.slab + (int64_t)L.nt * L.Mv + (int64_t)a * L.Mp;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.Mp; i += (int64_t)gridDim.x * blockDim.x)
    s += mom[i] * p[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[(int64_t)sl * kDotBlocks + blockIdx.x] = s;
}
__global__ void k_pmean_apply(LevelArgs L, const double* __restrict__ mean, double inv_vol, double* __restrict__ x,
                              int64_t ncells) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int sl = blockIdx.y, n = sl / L.nt, a = sl % L.nt;
  if (i >= ncells) return;
  x[(int64_t)n * L.slab + (int64_t)L.nt * L.Mv + (int64_t)a * L.Mp + i * L.C] -= mean[sl] * inv_vol;
}
hipError_t launch_project_pressure(const LevelArgs& L, const double* mom, double volume, double* x, double* partial,
                                   hipStream_t s) {
  int ns = L.N * L.nt;
  double* mean = partial + (int64_t)ns * kDotBlocks;
  k_pmean_partial<<<dim3(kDotBlocks, ns), 256, 0, s>>>(L, mom, x, partial);
  k_dot_final<<<(ns + 63) / 64, 64, 0, s>>>(partial, ns, mean);
  int64_t ncells = L.Mp / L.C;
  k_pmean_apply<<<dim3(nblk(ncells), ns), 256, 0, s>>>(L, mean, 1.0 / volume, x, ncells);
  return hipGetLastError();
}

// explicit instantiations
#define STMG_INST(T)                                                                                                \
  template hipError_t launch_apply<T>(const LevelArgs&, const double*, const T*, T, const T*, const T*, const T*,  \
                                      T*, int, T*, hipStream_t);                                                    \
  template hipError_t launch_vanka_factored<T>(const LevelArgs&, const T*, const T*, const T*, const T*, const T*, \
                                               const T*, T*, T, T*, hipStream_t);                                   \
  template hipError_t launch_vanka_dense<T>(const LevelArgs&, const T*, const T*, T*, T, hipStream_t);             \
  template hipError_t launch_prolongate_add<T>(const LevelArgs&, const LevelArgs&, const TransferDev&, const T*,   \
                                               const int*, const int*, const T*, const T*, const T*, T*, T*, T*,    \
                                               T*, hipStream_t);                                                    \
  template hipError_t launch_restrict<T>(const LevelArgs&, const LevelArgs&, const TransferDev&, const T*,         \
                                         const int*, const int*, const T*, const T*, const T*, T*, T*, T*, T*,      \
                                         hipStream_t);                                                              \
  template hipError_t launch_vanka_gather_only<T>(const LevelArgs&, const T*, T*, T, hipStream_t);                \
  template hipError_t launch_coarse<T>(int64_t, int64_t, int, int, const double*, const double*, const T*, T*,  \
                                        hipStream_t);                          \
  template hipError_t launch_fill<T>(T*, T, int64_t, hipStream_t);                                                  \
  template hipError_t launch_axpy<T>(T*, T, const T*, int64_t, hipStream_t);
STMG_INST(double)
STMG_INST(float)
#undef STMG_INST

}  // namespace stmg
