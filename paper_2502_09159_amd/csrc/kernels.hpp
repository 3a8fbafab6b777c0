// Device kernels of the hp space-time multigrid (gfx950).  Host-callable
// launchers; all work is enqueued on the given stream.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace stmg {

// Per-level sizes shared by the kernels.
struct LevelArgs {
  int d, n, q, Q, nn, nt, C, N, nloc;
  int64_t nodes, Mv, Mp, slab;
};

// Cell-local scratch E (every cell keeps its own copy of the nodes it
// shares; a gather kernel sums the copies of each node), per field
// f = (n nt + a) d + comp, in one of two layouts:
//  * operator (grid): a grid of (Q n)^d duplicated nodes, x fastest, in which
//    local node (ix, iy, iz) of cell (cx, cy, cz) sits at (cx Q + ix,
//    cy Q + iy, cz Q + iz), so that a row of global nodes reads contiguous
//    memory (the operator kernel writes whole cells per wave anyway);
//  * smoother (cell-major): cell by cell, local node i = ix + Q (iy + Q iz)
//    fastest, so that the one-cell-per-work-group smoother writes whole
//    cache lines (e_index).
// Spatial cells of a level (Mp < 2^31 is checked when the level is set up).
__device__ __forceinline__ int n_cells(const LevelArgs& L) { return (int)((unsigned)L.Mp / (unsigned)L.C); }
// Cell coordinates (x, y, z) of a cell index, x fastest (32-bit arithmetic).
__device__ __forceinline__ void cell_coords(const LevelArgs& L, int64_t cell, int (&cc)[3]) {
  const unsigned c = (unsigned)cell, n = (unsigned)L.n, r = c / n;
  cc[0] = (int)(c - r * n);
  cc[1] = L.d == 3 ? (int)(r % n) : (int)r;
  cc[2] = L.d == 3 ? (int)(r / n) : 0;
}
__device__ __forceinline__ int64_t e_index(const LevelArgs& L, int64_t field, int64_t cell, int i) {
  return (field * n_cells(L) + cell) * L.nloc + i;
}

// Small per-level tables, in the arithmetic type T, packed as
// [S (QxQ) | Dg (QxQ) | gx (Q) | gw (Q) | K (nt x nt) | phim1 (nt) | coef (nt) | psi (nloc x C)].
inline int table_size(int Q, int nt, int nloc, int C) { return 2 * Q * Q + 2 * Q + nt * nt + 2 * nt + nloc * C; }

// Operator: y = S x (mode 0) or y = b - S x (mode 1).  geo: per-cell Gauss
// point geometry (apply_geometry layout, in T).  Cell contributions to
// velocity nodes go to the cell-local scratch E (ncells * d * m * N values)
// and are summed per node in a fixed order (deterministic, no atomics).
template <typename T>
// gather = false runs the cell kernel only (E written, y's pressure rows
// written, velocity rows untouched): for timing.
// nper > 0 fixes the subintervals one wave walks through (clamped to [1, N]);
// 0 picks them so that the grid fills the chip.  variant: 0 and 1 the
// components as the outer loop of the cell kernel, 2 as the inner loop (3D
// FP32 only; elsewhere the outer loop is used).
hipError_t launch_apply(const LevelArgs& L, const T* geo, const T* tab, const T* x, const T* b, T* y, int mode,
                        T* E, hipStream_t s, bool gather = true, int nper = 0, int variant = 0);

// Slab right-hand side for time marching (Eq. (AlgSysTMS)) with lifted
// Dirichlet data, FP64: out = f - S_full g - C^1 v0 on free velocity rows and
// on pressure rows, 0 on Dirichlet rows.  S_full keeps every column of the
// operator; g supplies the Dirichlet values (its free entries are ignored);
// v0 (d x nodes, may be null) is the end value of the previous slab.  E is
// the level's cell scratch.
hipError_t launch_slab_rhs(const LevelArgs& L, const double* geo, const double* tab, const double* f,
                           const double* g, const double* v0, double* out, double* E, hipStream_t s);
// x = g on the Dirichlet velocity entries of a slab vector.
hipError_t launch_set_dirichlet(const LevelArgs& L, const double* g, double* x, hipStream_t s);

// Vanka correction with factored local inverses: x += omega D^-1 sum R^T A^-1 R r.
// Asw: A_s^{-1} of every cell in MFMA operand order (see vanka_swizzle_index),
// padded to mp = 16 ceil(m/16); E: cell-local scratch of ncells * d * m * N
// values (the velocity corrections, summed per node by a gather kernel).
template <typename T>
// gather = false runs the local solves only (E and the pressure updates): for timing.
// xzero: x holds no values yet and is taken as 0 (it is overwritten, not updated).
hipError_t launch_vanka_factored(const LevelArgs& L, const T* Asw, const T* Bm, const T* F, const T* Hinv,
                                 const T* coef, const T* r, T* x, T omega, T* E, hipStream_t s,
                                 bool gather = true, bool xzero = false);
// Row length of the device copies of F (per component: m rows of P) and of
// H^{-1} (P rows of P): P padded to a multiple of 4 values.
inline int vanka_row_pad(int P) { return (P + 3) / 4 * 4; }
// Position of A_s^{-1}[row][k] inside one cell's swizzled block (mp x mp):
// row tile t = row/16, k chunk kb = k/16, lane = row%16 + 16*((k%16)/4), slot k%4.
inline int64_t vanka_swizzle_index(int mp, int row, int k) {
  int t = row / 16, kb = k / 16, lane = row % 16 + 16 * ((k % 16) / 4), sl = k % 4;
  return (((int64_t)t * (mp / 16) + kb) * 64 + lane) * 4 + sl;
}
// Vanka correction with the temporally decoupled factors (one spatial Stokes
// block per eigenvalue of diag(c)^{-1} K: the real ones first, then one
// representative per complex-conjugate pair; the block count J and the number
// of real blocks follow from nt: J = (nt + 1) / 2, one real block iff nt is
// odd).  Per cell:
//   Aw: per block, Re (Ainv_j) then, for a complex block, Im (Ainv_j).  Both
//       are symmetric (Ainv_j inverts lambda_j M + A, M and A symmetric), so
//       each is stored as the upper triangle of its 16 x 16 tiles
//       (mp = 16 ceil(nloc / 16); vanka_sym_index);
//   Bm: C x d x nloc (as for the coupled factors);
//   Ft: [j][comp][i][row] with row = (re, im) of F_j[comp][i][l] for l < C,
//       padded to vanka_tdec_row(C) values;
//   Ht: [j][l][row] with row = (re, im) of Hinv_j[l][l'], padded likewise;
//   tw: per level, T (J x nt complex, (re, im)) then Wt (nt x J complex).
inline int vanka_tdec_row(int C) { return (2 * C + 3) / 4 * 4; }
// Position of entry (row, k), row / 16 <= k / 16, of a symmetric mp x mp block
// stored as its tiles (I, K), I <= K, row by row, each tile in MFMA operand
// order (lane = row%16 + 16*((k%16)/4), slot k%4, as vanka_swizzle_index).
// The kernel reads a tile below the diagonal as the transpose of its mirror.
inline int64_t vanka_sym_index(int mp, int row, int k) {
  const int nkb = mp / 16, I = row / 16, K = k / 16;
  const int up = I * nkb - I * (I - 1) / 2 + (K - I);
  const int lane = row % 16 + 16 * ((k % 16) / 4), sl = k % 4;
  return ((int64_t)up * 64 + lane) * 4 + sl;
}
inline int64_t vanka_tdec_aw(int nloc, int nt) {
  const int64_t nkb = (nloc + 15) / 16;
  return (int64_t)nt * nkb * (nkb + 1) / 2 * 256;  // 2 J - nreal = nt blocks of upper tiles
}
// diagonal: the diagonal Vanka (blocks lambda_j diag(M) + diag(A)): Aw holds
// nloc complex inverse diagonal entries per block (re, im) and Ft is unused.
template <typename T>
hipError_t launch_vanka_decoupled(const LevelArgs& L, const T* Aw, const T* Bm, const T* Ft, const T* Ht,
                                  const T* tw, const T* r, T* x, T omega, T* E, hipStream_t s,
                                  bool gather = true, bool xzero = false, bool diagonal = false);
// x_v += omega / valence * sum_cells E (the velocity half of a patch update);
// xzero: x_v holds no values yet, x_v = omega / valence * sum_cells E (0 on
// Dirichlet nodes).
template <typename T>
hipError_t launch_vanka_gather_only(const LevelArgs& L, const T* E, T* x, T omega, hipStream_t s,
                                    bool xzero = false);
// Same with one dense local inverse per cell.
template <typename T>
hipError_t launch_vanka_dense(const LevelArgs& L, const T* Ainv, const T* r, T* x, T omega, hipStream_t s);

// Transfers.  Tables (device): the 1D velocity embedding P1 (nnf x nnc) and
// its transpose P1T, each with the nonzero range [lo, hi) of every row and
// stored banded and transposed: P1[u * nnf + g] = P1(g, lo(g) + u) for u < 16
// (zero past the row), likewise P1T with nnc rows; E (npos x Cf x Cc); Pt
// (ntf x ntc) row-major.
struct TransferDev {
  int nnf, nnc, npos, ntf, ntc;
  bool time_change;
  int max_row_p1, max_row_p1t;  // longest nonzero range of a row of P1 / P1T
  int vt_p1 = 0, vt_p1t = 0;  // brick of the fused 3D prolongation / restriction (0: one pass per axis)
  int cap_p1[3] = {0, 0, 0}, cap_p1t[3] = {0, 0, 0};  // their largest staged brick extents
  const int* brk_p1 = nullptr;   // device: staged range (first, extent) of every brick, axis by axis
  const int* brk_p1t = nullptr;
};
// Plan of the fused 3D velocity transfer for the banded 1D matrix with row
// ranges [lo[o], hi[o]) and elements of `elem` bytes: picks the output brick
// whose staged input fits the LDS budget and returns its id (0 if none does:
// then the transfer runs as one pass per axis).  cap: largest staged extent
// per axis; brk: (first input node, extent) of every brick along x, then y,
// then z (bricks of the axis' own size).
int vtransfer_plan(const std::vector<int>& lo, const std::vector<int>& hi, int d, int max_row, bool restriction,
                   size_t elem, int* cap, std::vector<int>& brk);
template <typename T>
hipError_t launch_prolongate_add(const LevelArgs& F, const LevelArgs& Cs, const TransferDev& t,
                                 const T* P1, const int* rlo, const int* rhi, const T* E, const T* Pt,
                                 const T* xc, T* xf, T* tmp1, T* tmp2, T* tmp3, hipStream_t s);
template <typename T>
hipError_t launch_restrict(const LevelArgs& F, const LevelArgs& Cs, const TransferDev& t, const T* P1T,
                           const int* clo, const int* chi, const T* E, const T* Pt, const T* rf, T* bc, T* tmp1,
                           T* tmp2, T* tmp3, hipStream_t s);

// Coarse solve by forward substitution over the N subintervals:
// x_n = Dinv b_n - G x_{n-1}[last temporal dof, velocity] (FP64 matrices,
// Dinv slab x slab, G slab x Mv, row-major).
template <typename T>
hipError_t launch_coarse(int64_t slab, int64_t Mv, int nt, int N, const double* Dinv, const double* G, const T* b,
                         T* x, hipStream_t s);

// Vector helpers.
template <typename T>
hipError_t launch_fill(T* x, T v, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_axpy(T* y, T a, const T* x, int64_t n, hipStream_t s);  // y += a x
hipError_t launch_cast_d2f(const double* a, float* b, int64_t n, hipStream_t s);
hipError_t launch_cast_f2d(const float* a, double* b, int64_t n, hipStream_t s);
// Multi-dot: out[i] = V_i . w for i < nv (V rows of length n, stride ldv);
// partial buffer needs nv * 1024 doubles.
hipError_t launch_multidot(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* partial,
                           double* out, hipStream_t s);
// out[0] = a . b for vectors of type T (FP64 accumulation, fixed order);
// partial needs 1024 doubles.
template <typename T>
hipError_t launch_dot(const T* a, const T* b, int64_t n, double* partial, double* out, hipStream_t s);
// out[0..2] = <r, w>, <w, w>, <r, r> in one pass; partial needs 3 * 512 doubles.
template <typename T>
hipError_t launch_dot3(const T* r, const T* w, int64_t n, double* partial, double* out, hipStream_t s);
// One Arnoldi step of classical Gram-Schmidt with one reorthogonalisation,
// lagged by one step (two passes over the basis).  On entry V_0..V_{j-1} are
// final; if pending, u holds the previous step's vector after its first
// projection, with second-projection coefficients h2_prev (device) and norm
// 1/invb.  Pass 1 writes V_j = (u - V h2_prev) invb (if pending) and h1 =
// V_{0..j}^T w; pass 2 does w -= V h1 and writes h2n = (V^T w, |w|^2), nv + 1
// values with nv = j + 1.  Without a pending vector j must be 0 (V_0 final).
// partial needs (nv + 1) * 2048 doubles; nv <= kMaxFused.  Sums in a fixed
// order.
constexpr int kMaxFused = 64;
// w32 (may be null): receives w after pass 2 rounded to FP32.
hipError_t launch_lcgs2(double* V, int64_t ldv, int j, int pending, const double* u, const double* h2_prev,
                        double invb, double* w, int64_t n, double* partial, double* h1, double* h2n, float* w32,
                        hipStream_t s);
// w -= sum_i h_i V_i (h on device)
hipError_t launch_multi_axpy(double* w, const double* V, int64_t ldv, int nv, const double* h, int64_t n,
                             hipStream_t s);
// x += sum_i y_i Z_i (FP64 basis, or FP32 basis); assign: x = sum_i y_i Z_i
// (x not read)
hipError_t launch_combine(double* x, const double* Z, int64_t ldz, int nv, const double* y, int64_t n,
                          hipStream_t s, bool assign = false);
hipError_t launch_combine_f32(double* x, const float* Z, int64_t ldz, int nv, const double* y, int64_t n,
                              hipStream_t s, bool assign = false);
// scale: y = x * inv (and y32 = y rounded to FP32, when y32 is given)
hipError_t launch_scale_copy(double* y, const double* x, double inv, int64_t n, hipStream_t s,
                             float* y32 = nullptr);
// pressure mean removal per slice; mom: ncells x C moments; partial >= N nt 1024
hipError_t launch_project_pressure(const LevelArgs& L, const double* mom, double volume, double* x,
                                   double* partial, hipStream_t s);

}  // namespace stmg
