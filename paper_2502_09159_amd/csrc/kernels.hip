// Device kernels of the hp space-time multigrid for gfx950 (wave64).
//
// Data layout (Eq. (DefX)): X = (V_1, P_1, ..., V_N, P_N), V_n^a component-major
// over the global Gauss-Lobatto nodes, P_n^a cell-major over Legendre modes.
// Velocity contributions of the cells to the nodes they share go to a
// cell-local scratch E (one copy per cell) and are summed per node by gather
// kernels in a fixed order: no atomics, bit-reproducible results.  Only the
// dense-inverse smoother (a test path) adds into the nodes directly, race-free
// by 2^d-colouring the cells (cells of one colour share no node).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

#include <algorithm>

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

// Work groups are dispatched round-robin over the 8 XCDs (each with its own
// L2); remap the hardware block id so that every XCD works on one contiguous
// range of logical blocks (neighbouring cells share cache lines).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid64, int64_t nblocks64) {
  const unsigned bid = (unsigned)bid64, nblocks = (unsigned)nblocks64;  // grids stay below 2^32 blocks
  const unsigned q = nblocks >> 3, rem = nblocks & 7;
  const unsigned xcd = bid & 7, local = bid >> 3;
  return xcd < rem ? xcd * (q + 1) + local : rem * (q + 1) + (xcd - rem) * q + local;
}

}  // namespace

// =====================================================================
// Space-time operator (Eq. (GloSys) with Eq. (InAlg), (DefDtauh); M^tau
// diagonal).  For every temporal dof a of subinterval n:
//   y_v += K_ab M x_v[n,b] + c_a A_nu x_v[n,a] - c_a B^T x_p[n,a] - phi_a(-1) M x_v[n-1,k]
//   y_p += -c_a B x_v[n,a],      c_a = (tau/2) w_a.
// Mapping onto a wave: one cell per row of 16 lanes (a 4x4 grid of (x, y)
// node / Gauss-point positions, padded with zeros when Q = 3), the z
// direction held in registers (a pencil of Q values), four cells per wave.
// Sum-factorized 1D contractions run along x with quad-permute DPP, along y
// with row-rotate DPP and along z in registers: the loop has no LDS traffic
// besides small coefficient reads and no barriers.  A wave walks through the
// subintervals of its chunk and carries the end value of the previous
// subinterval (the jump term) in registers.  Geometry per Gauss point is
// precomputed: JxW, JxW J^{-1} and nu JxW J^{-1} J^{-T}.
// Velocity contributions go to the cell-local scratch E (summed per node by
// k_node_gather in a fixed order); pressure rows are written directly.
// =====================================================================
namespace {

// DPP lane permutations, each a bijection inside a group of 4 lanes (quad
// rotations) or inside a row of 16 lanes (rotations by multiples of 4).  The
// source lane of every permutation is read back on the device once per block,
// so the contraction coefficients never depend on the rotation direction.
constexpr int kQuadRot1 = 0x39, kQuadRot2 = 0x4E, kQuadRot3 = 0x93;  // quad_perm [1,2,3,0], [2,3,0,1], [3,0,1,2]
constexpr int kRowRot1 = 0x12C, kRowRot2 = 0x128, kRowRot3 = 0x124;  // row_ror 12, 8, 4
constexpr int kQuadSwap1 = 0xB1;

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)u);
  const unsigned hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// v from lane src (any lane of the wave)
__device__ __forceinline__ float lane_read(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_read(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Transposes, in place, a 16 x 16 tile held in MFMA operand order: lane
// i + 16 g, slot s holds entry [i][4 g + s]; afterwards it holds [4 g + s][i].
// With row = 4 r1 + r0 and column = 4 c1 + c0, entry [row][column] sits in
// lane bits (5:4, 3:2, 1:0) = (c1, r1, r0) and slot c0, and its transpose in
// (r1, c1, c0) and slot r0: a 4 x 4 transpose of (lane bits 1:0, slot) inside
// every quad of lanes (two butterfly stages, on lane bit 0 and lane bit 1),
// then the exchange of lane bits 5:4 and 3:2 across the wave.
template <typename T>
__device__ __forceinline__ void tile_transpose16(T (&v)[4], int lane) {
  const bool b0 = lane & 1, b1 = lane & 2;
  const T d0 = dpp<kQuadSwap1>(v[0]), d1 = dpp<kQuadSwap1>(v[1]);
  const T d2 = dpp<kQuadSwap1>(v[2]), d3 = dpp<kQuadSwap1>(v[3]);
  const T n0 = b0 ? d1 : v[0], n1 = b0 ? v[1] : d0, n2 = b0 ? d3 : v[2], n3 = b0 ? v[3] : d2;
  const T e0 = dpp<kQuadRot2>(n0), e1 = dpp<kQuadRot2>(n1), e2 = dpp<kQuadRot2>(n2), e3 = dpp<kQuadRot2>(n3);
  const T q[4] = {b1 ? e2 : n0, b1 ? e3 : n1, b1 ? n2 : e0, b1 ? n3 : e1};
  const int src = (((lane >> 2) & 3) << 4) | (((lane >> 4) & 3) << 2) | (lane & 3);
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) v[sl] = lane_read(q[sl], src);
}

// out = sum_m c[m] v(source lane of permutation m), along x (DIR 0) or y (DIR 1)
template <int DIR, typename T>
__device__ __forceinline__ T lane_contract(T v, const T* c) {
  if constexpr (__is_same(T, float)) {
    // FP32: one multiply and three FMAs whose first operand is read through
    // the permutation (the compiler does not fold a permutation into an FMA,
    // so it would spend a move on each).  The permutations are those of
    // kQuadRot1..3 / kRowRot1..3.  The no-ops keep two wait states between a
    // vector write of a register and a permuted read of it: v, written before
    // the block, and the result, which a permutation after it may read.
    float r;
    if constexpr (DIR == 0)
      asm("v_mul_f32 %0, %2, %1\n\ts_nop 1\n\t"
          "v_fmac_f32_dpp %0, %1, %3 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %1, %4 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %1, %5 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "s_nop 1"
          : "=&v"(r)
          : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    else
      asm("v_mul_f32 %0, %2, %1\n\ts_nop 1\n\t"
          "v_fmac_f32_dpp %0, %1, %3 row_ror:12 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %1, %4 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %1, %5 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "s_nop 1"
          : "=&v"(r)
          : "v"(v), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return r;
  } else if constexpr (DIR == 0)
    return c[0] * v + c[1] * dpp<kQuadRot1>(v) + c[2] * dpp<kQuadRot2>(v) + c[3] * dpp<kQuadRot3>(v);
  else
    return c[0] * v + c[1] * dpp<kRowRot1>(v) + c[2] * dpp<kRowRot2>(v) + c[3] * dpp<kRowRot3>(v);
}

// Sum over the 16 lanes of a row; every lane receives the sum.
template <typename T>
__device__ __forceinline__ T row_sum16(T v) {
  v += dpp<kRowRot2>(v);
  v += dpp<kRowRot3>(v);
  v += dpp<kQuadRot2>(v);
  v += dpp<kQuadSwap1>(v);
  return v;
}

// Offsets passed through an empty asm statement: the compiler may not hoist
// the small table reads that use them out of the subinterval loop (which
// would pin dozens of registers for the whole kernel).
__device__ __forceinline__ int opaque_v(int v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ int opaque_s(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

// FP32, all Q values of a pencil along x (DIR 0) or y (DIR 1) in one block:
// Q multiplies, then the three permuted FMAs of every value.  The first
// permuted read of an input comes Q instructions after the block starts (at
// least the two wait states a vector write needs before a permuted read of
// the same register), so only the results need the wait at the end.
template <int DIR, int ZP>
__device__ __forceinline__ void pencil_contract_f32(const float (&v)[ZP], float (&o)[ZP], const float (&c)[4]) {
  if constexpr (ZP == 4) {
    float r0, r1, r2, r3;
    if constexpr (DIR == 0)
      asm("v_mul_f32 %0, %8, %4\n\tv_mul_f32 %1, %8, %5\n\tv_mul_f32 %2, %8, %6\n\tv_mul_f32 %3, %8, %7\n\t"
          "v_fmac_f32_dpp %0, %4, %9 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %5, %9 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %6, %9 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %3, %7, %9 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %4, %10 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %5, %10 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %6, %10 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %3, %7, %10 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %4, %11 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %5, %11 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %6, %11 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %3, %7, %11 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "s_nop 1"
          : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
          : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    else
      asm("v_mul_f32 %0, %8, %4\n\tv_mul_f32 %1, %8, %5\n\tv_mul_f32 %2, %8, %6\n\tv_mul_f32 %3, %8, %7\n\t"
          "v_fmac_f32_dpp %0, %4, %9 row_ror:12 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %5, %9 row_ror:12 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %6, %9 row_ror:12 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %3, %7, %9 row_ror:12 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %4, %10 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %5, %10 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %6, %10 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %3, %7, %10 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %4, %11 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %5, %11 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %6, %11 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %3, %7, %11 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "s_nop 1"
          : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
          : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
  } else {
    float r0, r1, r2;
    if constexpr (DIR == 0)
      asm("v_mul_f32 %0, %6, %3\n\tv_mul_f32 %1, %6, %4\n\tv_mul_f32 %2, %6, %5\n\t"
          "v_fmac_f32_dpp %0, %3, %7 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %4, %7 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %5, %7 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %3, %8 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %4, %8 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %5, %8 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %3, %9 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %4, %9 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %5, %9 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "s_nop 1"
          : "=&v"(r0), "=&v"(r1), "=&v"(r2)
          : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    else
      asm("v_mul_f32 %0, %6, %3\n\tv_mul_f32 %1, %6, %4\n\tv_mul_f32 %2, %6, %5\n\t"
          "v_fmac_f32_dpp %0, %3, %7 row_ror:12 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %4, %7 row_ror:12 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %5, %7 row_ror:12 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %3, %8 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %4, %8 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %5, %8 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %0, %3, %9 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %1, %4, %9 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "v_fmac_f32_dpp %2, %5, %9 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
          "s_nop 1"
          : "=&v"(r0), "=&v"(r1), "=&v"(r2)
          : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    o[0] = r0; o[1] = r1; o[2] = r2;
  }
}

// Pencil contraction with 1D matrix `mat` (0: S, 1: Dg, 2: S^T, 3: Dg^T) along
// direction DIR of a cell.  x / y: per-lane coefficients cxy[co + m] in LDS
// (co = mat * 16 + position * 4); z: the Q x Q matrices in global memory
// (uniform reads), tS / tDg.
template <int DIR, int Q, int ZP, typename T>
__device__ __forceinline__ void pencil(const T (&v)[ZP], T (&o)[ZP], int mat, const T* cxy, int co,
                                       const T* __restrict__ tz) {
  if constexpr (DIR == 2) {
    const T* M = tz + opaque_s((mat & 1) * Q * Q);
#pragma unroll
    for (int z = 0; z < ZP; ++z) {
      T s = 0;
#pragma unroll
      for (int t = 0; t < ZP; ++t) s += (mat < 2 ? M[z * Q + t] : M[t * Q + z]) * v[t];
      o[z] = s;
    }
  } else {
    const int c0 = opaque_v(co);
    T cc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) cc[m] = cxy[c0 + m];
    // one block per pencil on Q2 levels.  On Q3 levels the four inputs and
    // four results it holds at once cost the fourth wave per SIMD; capped to
    // four waves it spilled and ran 0.39-0.42 ms against 0.33-0.36 ms with one
    // block per value (cell kernel, C5 finest level)
    if constexpr (__is_same(T, float) && ZP == 3) {
      pencil_contract_f32<DIR, ZP>(v, o, cc);
    } else {
#pragma unroll
      for (int z = 0; z < ZP; ++z) o[z] = lane_contract<DIR>(v[z], cc);
    }
  }
}

}  // namespace

// The pressure modes of degree R in 3D as products of shifted Legendre
// factors P_a(x) P_b(y) P_c(z), in the library's mode order (total degree
// 0..R, then the x exponent largest first, then the y exponent): for each
// mode, the index of (a, b) among the pairs with a + b <= R (by a + b, then a
// largest first) and c.
struct PMode {
  int pair, c;
};
template <int R>
struct PModes {
  PMode m[(R + 1) * (R + 2) * (R + 3) / 6];
};
template <int R>
__host__ __device__ constexpr PModes<R> pmodes() {
  PModes<R> t{};
  int idx = 0;
  for (int d = 0; d <= R; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) t.m[idx++] = PMode{(a + b) * (a + b + 1) / 2 + b, d - a - b};
  return t;
}

// FULL: every column of the operator, Dirichlet ones included (x is read at
// every node), and for the first subinterval the jump term takes the end
// value v0 of the previous slab (d x nodes, or none): y = b - S_full x - C^1 v0
// on free rows, the lifting of inhomogeneous Dirichlet data (Eq. (AlgSysTMS)).
// CI (3D): the components are the inner loop, so the pressure at the Gauss
// points, the continuity-row reduction and its store are done once per
// (subinterval, temporal dof) instead of once per component; all components'
// metric, nodal values and jump values stay in registers.
template <typename T, int D, int Q, int NT, bool FULL = false, bool CI = false>
__global__ __launch_bounds__(256) void k_apply(LevelArgs L, const T* __restrict__ geo, const T* __restrict__ tab,
                                               const T* __restrict__ x, const T* __restrict__ b,
                                               T* __restrict__ y, T* __restrict__ E, int mode, int nper,
                                               const T* __restrict__ v0 = nullptr) {
  constexpr int ZP = D == 3 ? Q : 1;
  constexpr int NL = D == 3 ? Q * Q * Q : Q * Q;
  constexpr int NG = 1 + D * D + D * (D + 1) / 2;
  constexpr int NS = D * (D + 1) / 2;
  constexpr int C = D == 3 ? (Q - 1) * Q * (Q + 1) / 6 : (Q - 1) * Q / 2;
  __shared__ __align__(16) T sCX[64];
  __shared__ __align__(16) T sCY[64];
  __shared__ T sPsi[D == 3 ? 1 : 16 * ZP * C];  // 2D only
  __shared__ int sSrc[2][4][4];
  const int tid = threadIdx.x, lane16 = tid & 15, qx = lane16 & 3, qy = lane16 >> 2;
  const T* tS = tab;
  const T* tDg = tS + Q * Q;
  const T* tK = tDg + Q * Q + 2 * Q;
  const T* tphi = tK + NT * NT;
  const T* tcoef = tphi + NT;
  const T* tpsi = tcoef + NT;

  // ---- source lanes of the DPP permutations (wave 0, all lanes active)
  if (tid < 64) {
    const int sx1 = dpp_i<kQuadRot1>(qx), sx2 = dpp_i<kQuadRot2>(qx), sx3 = dpp_i<kQuadRot3>(qx);
    const int sy1 = dpp_i<kRowRot1>(lane16) >> 2, sy2 = dpp_i<kRowRot2>(lane16) >> 2,
              sy3 = dpp_i<kRowRot3>(lane16) >> 2;
    if (tid < 16 && qy == 0) {
      sSrc[0][0][qx] = qx; sSrc[0][1][qx] = sx1; sSrc[0][2][qx] = sx2; sSrc[0][3][qx] = sx3;
    }
    if (tid < 16 && qx == 0) {
      sSrc[1][0][qy] = qy; sSrc[1][1][qy] = sy1; sSrc[1][2][qy] = sy2; sSrc[1][3][qy] = sy3;
    }
  }
  __syncthreads();
  auto mat_el = [&](int mat, int i, int t) -> T {
    if (i >= Q || t >= Q) return T(0);
    const T* M = (mat & 1) ? tDg : tS;
    return mat < 2 ? M[i * Q + t] : M[t * Q + i];
  };
  if (tid < 64) {
    const int mat = tid >> 4, i = (tid >> 2) & 3, m = tid & 3;
    sCX[tid] = mat_el(mat, i, sSrc[0][m][i]);
    sCY[tid] = mat_el(mat, i, sSrc[1][m][i]);
  }
  // sPsi[(z C + l) 16 + lane16]: the lanes of a row read consecutive words (no bank conflicts)
  for (int t = tid; t < (D == 3 ? 0 : 16 * ZP * C); t += blockDim.x) {
    const int ll = t % 16, l = (t / 16) % C, z = t / (16 * C), px = ll & 3, py = ll >> 2;
    sPsi[t] = (px < Q && py < Q) ? tpsi[(px + Q * py + Q * Q * z) * C + l] : T(0);
  }
  __syncthreads();

  // ---- this lane's cell, chunk of subintervals and nodes
  const int64_t ncells = L.Mp / C;
  const int64_t nbx = gridDim.x;
  const int64_t lb = xcd_remap(blockIdx.x + nbx * blockIdx.y, nbx * gridDim.y);
  const int64_t cid = (lb % nbx) * 16 + (tid >> 4);
  const int n0 = (int)(lb / nbx) * nper;
  const int n1 = min(L.N, n0 + nper);
  const bool cvalid = cid < ncells;
  const bool lvalid = cvalid && qx < Q && qy < Q;
  const int64_t cell = cvalid ? cid : 0;
  int ccs[3];
  cell_coords(L, cell, ccs);
  const int cc0 = ccs[0], cc1 = ccs[1], cc2 = ccs[2];
  const int gxn = cc0 * L.q + qx, gyn = cc1 * L.q + qy;
  const bool fxy = lvalid && gxn > 0 && gxn < L.nn - 1 && gyn > 0 && gyn < L.nn - 1;
  int gnd[ZP];  // node index (< 2^31: checked on the host)
  bool fre[ZP];
#pragma unroll
  for (int z = 0; z < ZP; ++z) {
    const int gzn = cc2 * L.q + z;
    gnd[z] = gxn + L.nn * (gyn + (D == 3 ? L.nn * gzn : 0));
    fre[z] = fxy && (D == 2 || (gzn > 0 && gzn < L.nn - 1));
  }
  const T* gc = geo + (cell * NG * 16 + lane16) * ZP;  // geo[cell][f][lane16][z]
  // E: per field (n, a, comp) a grid of (Q n)^d duplicated nodes (each cell
  // keeps its own copy of shared nodes), x fastest
  const int W = Q * L.n;
  const int64_t NE = D == 3 ? (int64_t)W * W * W : (int64_t)W * W;
  T* Ec = E + (cc0 * Q + qx) + (int64_t)W * (cc1 * Q + qy) + (D == 3 ? (int64_t)W * W * cc2 * Q : 0);
  const int po = lane16;  // this lane's column of the psi table
  // 3D: the pressure and continuity rows use the factors of the modes
  // (pmodes): pxy[pair] is this lane's (x, y) factor at its Gauss point (0 on
  // padded lanes), pz[c][z] the z factor at Gauss point z, both read from the
  // psi table at the modes (a, b, 0) and (0, 0, c) (P_0 = 1).  A pressure value
  // then costs C + (R + 1) ZP multiply-adds per lane instead of C ZP.
  constexpr int R = Q - 2, NPAIR = (R + 1) * (R + 2) / 2;
  constexpr PModes<R> PM = pmodes<R>();
  T pxy[D == 3 ? NPAIR : 1], pz[D == 3 ? R + 1 : 1][ZP];
  if constexpr (D == 3) {
    const bool inq = qx < Q && qy < Q;
    const int pxyi = min(qx, Q - 1) + Q * min(qy, Q - 1);
#pragma unroll
    for (int l = 0; l < C; ++l) {
      const PMode m = PM.m[l];
      if (m.c == 0) pxy[m.pair] = inq ? tpsi[pxyi * C + l] : T(0);
      if (m.pair == 0)
#pragma unroll
        for (int z = 0; z < ZP; ++z) pz[m.c][z] = tpsi[(Q * Q * z) * C + l];
    }
  }
  // pressure of the C modes pl at this lane's Gauss points
  auto pressure_at = [&](const T (&pl)[C], T (&pres)[ZP], int pr) {
    if constexpr (D == 3) {
      T A[R + 1];
#pragma unroll
      for (int c = 0; c <= R; ++c) A[c] = 0;
#pragma unroll
      for (int l = 0; l < C; ++l) {
        const PMode m = PM.m[l];
        A[m.c] += pl[l] * pxy[m.pair];
      }
#pragma unroll
      for (int z = 0; z < ZP; ++z) {
        T v = 0;
#pragma unroll
        for (int c = 0; c <= R; ++c) v += pz[c][z] * A[c];
        pres[z] = v;
      }
    } else {
#pragma unroll
      for (int z = 0; z < ZP; ++z) {
        T v = 0;
#pragma unroll
        for (int l = 0; l < C; ++l) v += sPsi[pr + (z * C + l) * 16] * pl[l];
        pres[z] = v;
      }
    }
  };
  // continuity rows: sum over the cell's Gauss points of psi_l dv, mode l in lane l
  auto continuity = [&](const T (&dv)[ZP], int pr) -> T {
    T mine = 0;
    if constexpr (D == 3) {
      T B[R + 1];
#pragma unroll
      for (int c = 0; c <= R; ++c) {
        T v = 0;
#pragma unroll
        for (int z = 0; z < ZP; ++z) v += pz[c][z] * dv[z];
        B[c] = v;
      }
#pragma unroll
      for (int l = 0; l < C; ++l) {
        const PMode m = PM.m[l];
        const T v = row_sum16(pxy[m.pair] * B[m.c]);
        if (lane16 == l) mine = v;
      }
    } else {
#pragma unroll
      for (int l = 0; l < C; ++l) {
        T v = 0;
#pragma unroll
        for (int z = 0; z < ZP; ++z) v += sPsi[pr + (z * C + l) * 16] * dv[z];
        v = row_sum16(v);
        if (lane16 == l) mine = v;
      }
    }
    return mine;
  };

  // nodal values of (n, temporal dof bb, comp) interpolated to the Gauss
  // points (n = -1: the previous slab's end value v0, FULL only)
  auto interp = [&](int n, int bb, int comp, T (&uq)[ZP]) {
    T v[ZP], w[ZP];
    const T* xs = (FULL && n < 0) ? v0 + (int64_t)comp * L.nodes
                                  : x + (int64_t)n * L.slab + (int64_t)bb * L.Mv + (int64_t)comp * L.nodes;
    // FP32: read unconditionally (node 0 stands in for lanes without a free
    // node), so that no load waits behind a per-lane branch (FP64 ran 6%
    // slower so, and keeps the predicated loads)
#pragma unroll
    for (int z = 0; z < ZP; ++z) {
      const bool rd = FULL ? lvalid : fre[z];
      if constexpr (sizeof(T) == 4) {
        const T t = xs[rd ? gnd[z] : 0];
        v[z] = rd ? t : T(0);
      } else {
        v[z] = rd ? xs[gnd[z]] : T(0);
      }
    }
    pencil<0, Q, ZP>(v, w, 0, sCX, qx * 4, tS);
    if constexpr (D == 3) {
      pencil<1, Q, ZP>(w, v, 0, sCY, qy * 4, tS);
      pencil<2, Q, ZP>(v, uq, 0, sCX, 0, tS);
    } else {
      pencil<1, Q, ZP>(w, uq, 0, sCY, qy * 4, tS);
    }
  };

  if constexpr (CI) {
    static_assert(D == 3, "components-inner evaluation is for 3D levels");
    // geometry: JxW, nu JxW J^-1 J^-T, and every column of JxW J^-1
    T jw[ZP], gm[NS][ZP], ja[D][D][ZP];  // ja[comp][j][z]
#pragma unroll
    for (int z = 0; z < ZP; ++z) {
      jw[z] = gc[z];
#pragma unroll
      for (int comp = 0; comp < D; ++comp)
#pragma unroll
        for (int j = 0; j < D; ++j) ja[comp][j][z] = gc[(1 + j * D + comp) * 16 * ZP + z];
#pragma unroll
      for (int t = 0; t < NS; ++t) gm[t][z] = gc[(1 + D * D + t) * 16 * ZP + z];
    }
    T up[D][ZP];
#pragma unroll
    for (int comp = 0; comp < D; ++comp) {
      if (n0 > 0 && n0 < n1) interp(n0 - 1, NT - 1, comp, up[comp]);
      else
#pragma unroll
        for (int z = 0; z < ZP; ++z) up[comp][z] = 0;
    }
    for (int n = n0; n < n1; ++n) {
      T uq[D][NT][ZP];
#pragma unroll
      for (int comp = 0; comp < D; ++comp)
#pragma unroll
        for (int bb = 0; bb < NT; ++bb) interp(n, bb, comp, uq[comp][bb]);
      // temporal dofs one at a time; uq[comp] is rotated so that uq[comp][0]
      // holds dof a and uq[comp][j] dof (a + j) mod NT
#pragma unroll 1
      for (int a = 0; a < NT; ++a) {
        const T ca = tcoef[a];
        const int64_t prow = (int64_t)n * L.slab + (int64_t)NT * L.Mv + (int64_t)a * L.Mp + cell * C;
        const T prev_in = mode ? b[prow + min(lane16, C - 1)] : T(0);
        T pres[ZP];
        {
          const T* ps = x + prow + opaque_v(0);
          T pl[C];
#pragma unroll
          for (int l = 0; l < C; ++l) {
            const T v = ps[l];
            pl[l] = cvalid ? v : T(0);
          }
          pressure_at(pl, pres, opaque_v(po));
        }
        T dvs[ZP];
#pragma unroll
        for (int z = 0; z < ZP; ++z) dvs[z] = 0;
#pragma unroll
        for (int comp = 0; comp < D; ++comp) {
          T Zq[ZP];
#pragma unroll
          for (int z = 0; z < ZP; ++z) {
            T w = -tphi[a] * up[comp][z];
#pragma unroll
            for (int j = 0; j < NT; ++j) {
              const int bb = a + j < NT ? a + j : a + j - NT;
              w += tK[a * NT + bb] * uq[comp][j][z];
            }
            Zq[z] = w * jw[z];
          }
          T g[3][ZP];
          pencil<0, Q, ZP>(uq[comp][0], g[0], 1, sCX, 16 + qx * 4, tS);
          pencil<1, Q, ZP>(uq[comp][0], g[1], 1, sCY, 16 + qy * 4, tS);
          pencil<2, Q, ZP>(uq[comp][0], g[2], 1, sCX, 0, tS);
#pragma unroll
          for (int z = 0; z < ZP; ++z) {
            T gr[D];
#pragma unroll
            for (int j = 0; j < D; ++j) gr[j] = g[j][z];
            T dsum = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
              T s = 0;
#pragma unroll
              for (int k = 0; k < D; ++k) {
                const int t = j <= k ? j * D - j * (j - 1) / 2 + (k - j) : k * D - k * (k - 1) / 2 + (j - k);
                s += gm[t][z] * gr[k];
              }
              g[j][z] = ca * (s - pres[z] * ja[comp][j][z]);
              dsum += ja[comp][j][z] * gr[j];
            }
            dvs[z] -= ca * dsum;
          }
          T t1[ZP];
          pencil<0, Q, ZP>(g[0], t1, 3, sCX, 48 + qx * 4, tS);
#pragma unroll
          for (int z = 0; z < ZP; ++z) Zq[z] += t1[z];
          pencil<1, Q, ZP>(g[1], t1, 3, sCY, 48 + qy * 4, tS);
#pragma unroll
          for (int z = 0; z < ZP; ++z) Zq[z] += t1[z];
          pencil<2, Q, ZP>(g[2], t1, 3, sCX, 0, tS);
#pragma unroll
          for (int z = 0; z < ZP; ++z) Zq[z] += t1[z];
          pencil<0, Q, ZP>(Zq, t1, 2, sCX, 32 + qx * 4, tS);
          pencil<1, Q, ZP>(t1, Zq, 2, sCY, 32 + qy * 4, tS);
          pencil<2, Q, ZP>(Zq, t1, 2, sCX, 0, tS);
          if (lvalid) {
            T* Eo = Ec + ((int64_t)(n * NT + a) * D + comp) * NE;
#pragma unroll
            for (int z = 0; z < ZP; ++z) Eo[(int64_t)W * W * z] = t1[z];
          }
        }
        // continuity rows of dof a, all components at once
        {
          const T mine = continuity(dvs, opaque_v(po));
          if (cvalid && lane16 < C) y[prow + lane16] = mode ? prev_in - mine : mine;
        }
#pragma unroll
        for (int comp = 0; comp < D; ++comp)
#pragma unroll
          for (int z = 0; z < ZP; ++z) {
            const T first = uq[comp][0][z];
#pragma unroll
            for (int j = 0; j + 1 < NT; ++j) uq[comp][j][z] = uq[comp][j + 1][z];
            uq[comp][NT - 1][z] = first;
          }
      }
#pragma unroll
      for (int comp = 0; comp < D; ++comp)
#pragma unroll
        for (int z = 0; z < ZP; ++z) up[comp][z] = uq[comp][NT - 1][z];
    }
    return;
  }

#pragma unroll 1
  for (int comp = 0; comp < D; ++comp) {
    // geometry of this component: JxW, nu JxW J^-1 J^-T, column comp of JxW J^-1
    T jw[ZP], gm[NS][ZP], ja[D][ZP];
#pragma unroll
    for (int z = 0; z < ZP; ++z) {
      jw[z] = gc[z];
#pragma unroll
      for (int j = 0; j < D; ++j) ja[j][z] = gc[(1 + j * D + comp) * 16 * ZP + z];
#pragma unroll
      for (int t = 0; t < NS; ++t) gm[t][z] = gc[(1 + D * D + t) * 16 * ZP + z];
    }
    T up[ZP];
    if (n0 > 0 && n0 < n1) interp(n0 - 1, NT - 1, comp, up);
    else if (FULL && n0 == 0 && v0 != nullptr) interp(-1, NT - 1, comp, up);
    else
#pragma unroll
      for (int z = 0; z < ZP; ++z) up[z] = 0;

    for (int n = n0; n < n1; ++n) {
      T uq[NT][ZP];
#pragma unroll
      for (int bb = 0; bb < NT; ++bb) interp(n, bb, comp, uq[bb]);
      // temporal dofs one at a time (not unrolled: bounded register use); uq is
      // rotated so that uq[0] holds dof a and uq[j] holds dof (a + j) mod NT
#pragma unroll 1
      for (int a = 0; a < NT; ++a) {
        const T ca = tcoef[a];
        // the continuity row this lane accumulates into at the end of the step,
        // read now (clamped to a row of this cell, so always in bounds) so that
        // its latency overlaps the step
        const int64_t prow = (int64_t)n * L.slab + (int64_t)NT * L.Mv + (int64_t)a * L.Mp + cell * C;
        const T prev_in = (comp > 0 ? y : (mode ? b : y))[prow + min(lane16, C - 1)];
        // pressure of dof a at the Gauss points (read unconditionally: cell is
        // clamped to 0 past the last cell, and those lanes take zeros)
        T pres[ZP];
        {
          const T* ps = x + prow + opaque_v(0);
          T pl[C];
#pragma unroll
          for (int l = 0; l < C; ++l) {
            const T v = ps[l];
            pl[l] = cvalid ? v : T(0);
          }
          pressure_at(pl, pres, opaque_v(po));
        }
        T Zq[ZP];
#pragma unroll
        for (int z = 0; z < ZP; ++z) {
          T w = -tphi[a] * up[z];
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const int bb = a + j < NT ? a + j : a + j - NT;
            w += tK[a * NT + bb] * uq[j][z];
          }
          Zq[z] = w * jw[z];
        }
        T g[3][ZP];
        pencil<0, Q, ZP>(uq[0], g[0], 1, sCX, 16 + qx * 4, tS);
        pencil<1, Q, ZP>(uq[0], g[1], 1, sCY, 16 + qy * 4, tS);
        if constexpr (D == 3) pencil<2, Q, ZP>(uq[0], g[2], 1, sCX, 0, tS);
        T dv[ZP];
#pragma unroll
        for (int z = 0; z < ZP; ++z) {
          T gr[D];
#pragma unroll
          for (int j = 0; j < D; ++j) gr[j] = g[j][z];
          T dsum = 0;
#pragma unroll
          for (int j = 0; j < D; ++j) {
            T s = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
              const int t = j <= k ? j * D - j * (j - 1) / 2 + (k - j) : k * D - k * (k - 1) / 2 + (j - k);
              s += gm[t][z] * gr[k];
            }
            g[j][z] = ca * (s - pres[z] * ja[j][z]);
            dsum += ja[j][z] * gr[j];
          }
          dv[z] = -ca * dsum;
        }
        // test with the reference gradients (transposed collocation derivative)
        T t1[ZP];
        pencil<0, Q, ZP>(g[0], t1, 3, sCX, 48 + qx * 4, tS);
#pragma unroll
        for (int z = 0; z < ZP; ++z) Zq[z] += t1[z];
        pencil<1, Q, ZP>(g[1], t1, 3, sCY, 48 + qy * 4, tS);
#pragma unroll
        for (int z = 0; z < ZP; ++z) Zq[z] += t1[z];
        if constexpr (D == 3) {
          pencil<2, Q, ZP>(g[2], t1, 3, sCX, 0, tS);
#pragma unroll
          for (int z = 0; z < ZP; ++z) Zq[z] += t1[z];
        }
        // back to the nodes: transposed interpolation
        pencil<0, Q, ZP>(Zq, t1, 2, sCX, 32 + qx * 4, tS);
        if constexpr (D == 3) {
          pencil<1, Q, ZP>(t1, Zq, 2, sCY, 32 + qy * 4, tS);
          pencil<2, Q, ZP>(Zq, t1, 2, sCX, 0, tS);
        } else {
          pencil<1, Q, ZP>(t1, Zq, 2, sCY, 32 + qy * 4, tS);
#pragma unroll
          for (int z = 0; z < ZP; ++z) t1[z] = Zq[z];
        }
        if (lvalid) {
          T* Eo = Ec + ((int64_t)(n * NT + a) * D + comp) * NE;
#pragma unroll
          for (int z = 0; z < ZP; ++z) Eo[(int64_t)W * W * z] = t1[z];
        }
        // continuity rows of dof a: y_p[l] (+)= -c_a sum_q psi_l(q) JxW d_comp u_a(q),
        // accumulated over the components in a fixed order
        {
          const T mine = continuity(dv, opaque_v(po));
          if (cvalid && lane16 < C) {
            const T prev = comp > 0 || mode ? prev_in : T(0);
            y[prow + lane16] = mode ? prev - mine : prev + mine;
          }
        }
        // rotate: uq[j] <- uq[j + 1]
#pragma unroll
        for (int z = 0; z < ZP; ++z) {
          const T first = uq[0][z];
#pragma unroll
          for (int j = 0; j + 1 < NT; ++j) uq[j][z] = uq[j + 1][z];
          uq[NT - 1][z] = first;
        }
      }
      // after NT rotations uq is back in order; the last dof feeds the next jump term
#pragma unroll
      for (int z = 0; z < ZP; ++z) up[z] = uq[NT - 1][z];
    }
  }
}

// Node gathers over the duplicated-grid scratch E.  One thread owns the q
// nodes g = q c + j (j < q) of cell interval c along x in one row (y, z) of one
// field; the thread of the last interval also owns the last node of the row.
// Node g has duplicated index Q c + j in its own cell and, for j = 0 and c > 0,
// Q c - 1 in the cell below; the same holds along y and z (row-uniform).
// Launch: 256 threads = XW intervals x (256 / XW) rows (XW = 2^lxw, the
// smallest power of two >= n, at most 64), grid (ceil(n / XW),
// ceil(nn / rows) nn (3D) or ceil(nn / rows) (2D), d nt N fields).
//   KIND 0 (operator): y = sum (mode 0) or b - sum (mode 1); Dirichlet rows identity
//   KIND 1 (smoother): x += omega / valence * sum; Dirichlet nodes unchanged
//                      (mode 1: x starts at 0, so x = omega / valence * sum and 0)
template <typename T, int D, int QQ, int KIND, int mode>
__global__ __launch_bounds__(256) void k_node_gather(LevelArgs L, const T* __restrict__ E, const T* __restrict__ xin,
                                                     const T* __restrict__ b, T* __restrict__ out, T omega,
                                                     int lxw) {
  constexpr int q = QQ - 1;
  // logical block.  Smoother (cell-major E): consecutive blocks share the
  // copies of shared nodes (the two z-layers in a cache line of a cell, rows
  // straddling two blocks), so they are kept on one XCD and its L2: the
  // finest level's gather then fetches its E and x once instead of twice.
  // The operator's grid layout reads whole rows and measured 2-5% slower so.
  const int64_t gxy = (int64_t)gridDim.x * gridDim.y;
  const int64_t hw = blockIdx.x + gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  const int64_t lb = KIND == 1 ? xcd_remap(hw, gxy * gridDim.z) : hw;
  const int bx = (int)(lb % gridDim.x), by = (int)((lb / gridDim.x) % gridDim.y);
  // the work group's XW intervals x rows; smoother on Q3 levels with XW >=
  // 16: a wave takes 16 intervals x 4 consecutive rows, the 4 rows of an
  // interval in consecutive lanes, so that the rows of a cell's z-layer in the
  // cell-major scratch are read by neighbouring lanes (2-4% faster at C5; 5%
  // slower on Q2 levels, whose 3-row z-layers straddle the 4-row groups)
  int tc = (int)(threadIdx.x & ((1 << lxw) - 1)), tr = (int)(threadIdx.x >> lxw);
  if (KIND == 1 && QQ == 4 && lxw >= 4) {
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6), wc = 1 << (lxw - 4);
    tc = (w % wc) * 16 + (lane >> 2);
    tr = (w / wc) * 4 + (lane & 3);
  }
  const int c = (bx << lxw) + tc;
  const int rows = 256 >> lxw, nyb = (L.nn + rows - 1) / rows;
  const int gy = (D == 3 ? by % nyb : by) * rows + tr;
  const int gz = D == 3 ? by / nyb : 0;
  if (c >= L.n || gy >= L.nn) return;
  const int64_t field = lb / gxy;  // (n nt + a) D + comp
  const int comp = (int)(field % D);
  const int64_t fa = field / D;
  const int64_t row0 = (fa / L.nt) * L.slab + (fa % L.nt) * L.Mv + (int64_t)comp * L.nodes +
                       (int64_t)L.nn * (gy + (int64_t)L.nn * gz);
  const bool brow = gy == 0 || gy == L.nn - 1 || (D == 3 && (gz == 0 || gz == L.nn - 1));
  const int g0 = q * c;
  const bool last = c == L.n - 1;
  if (brow) {  // every node of a boundary row is a Dirichlet node
    if (KIND == 0 || mode) {
#pragma unroll
      for (int j = 0; j < q + 1; ++j) {
        if (j == q && !last) break;
        const int64_t id = row0 + g0 + j;
        if (KIND == 0) out[id] = mode == 2 ? T(0) : (mode ? b[id] - xin[id] : xin[id]);
        else out[id] = T(0);
      }
    }
    return;
  }
  // KIND 0 reads the operator's grid layout, KIND 1 the smoother's cell-major one
  constexpr bool CM = KIND == 1;
  constexpr int NLQ = D == 3 ? QQ * QQ * QQ : QQ * QQ;
  const int W = QQ * L.n;
  const int64_t NE = CM ? (int64_t)n_cells(L) * NLQ : (D == 3 ? (int64_t)W * W * W : (int64_t)W * W);
  const T* Ef = E + field * NE;
  const int ny = (gy % q == 0) ? 2 : 1, nz = D == 3 ? ((gz % q == 0) ? 2 : 1) : 1;
  const int dy = gy + gy / q, dz = gz + gz / q;
  // the values the outputs need, read first (node q of the row start belongs
  // to the next thread unless this is the last one: read anyway)
  T bv[q + 1], xv[q + 1];
#pragma unroll
  for (int j = 0; j < q + 1; ++j) {
    const int64_t id = row0 + g0 + j;
    if (KIND == 0 && mode) bv[j] = b[id];  // (modes 1 and 2)
    if (KIND == 1 && !mode) xv[j] = out[id];
  }
  // Dirichlet nodes of the row (x = 0 and x = 1): the operator copies x there
  const T xd0 = KIND == 0 ? xin[row0] : T(0), xd1 = KIND == 0 ? xin[row0 + L.nn - 1] : T(0);
  // the copies of the thread's nodes, summed in a fixed order (u, v): own
  // cell, then the cell below along x.  In the grid layout every copy is read
  // unconditionally (one a node does not have is read from its own row and
  // weighted out), so that all loads are in flight together (a load under a
  // branch makes the compiler wait for it); in the cell-major layout such
  // extra reads would each touch a line per lane, so only the needed ones are made.
  T own[q], below = T(0);
#pragma unroll
  for (int j = 0; j < q; ++j) own[j] = T(0);
  auto row_ptr = [&](int uu, int vv) -> const T* {  // x-row (dy - vv, dz - uu) of cell c
    if constexpr (CM) {
      const int DY = dy - vv, DZ = D == 3 ? dz - uu : 0;
      const int64_t cellc = c + (int64_t)L.n * ((DY / QQ) + (D == 3 ? (int64_t)L.n * (DZ / QQ) : 0));
      return Ef + cellc * NLQ + ((D == 3 ? (DZ % QQ) * QQ : 0) + DY % QQ) * QQ;
    } else {
      return Ef + (D == 3 ? (int64_t)(dz - uu) * W * W : 0) + (int64_t)(dy - vv) * W + (int64_t)QQ * c;
    }
  };
  auto read_row = [&](const T* er, T (&ev)[q]) {
    if constexpr (QQ == 4 && sizeof(T) == 4) {  // 16-byte aligned
      const float4 t4 = *reinterpret_cast<const float4*>(er);
      ev[0] = t4.x; ev[1] = t4.y; ev[2] = t4.z;
    } else if constexpr (QQ == 4) {
      const double2 t0 = *reinterpret_cast<const double2*>(er);
      ev[0] = t0.x; ev[1] = t0.y; ev[2] = er[2];
    } else {
#pragma unroll
      for (int j = 0; j < q; ++j) ev[j] = er[j];
    }
  };
  // el - 1: the last node of the row in cell c - 1
  auto left_ptr = [&](const T* er) -> const T* { return CM ? er - NLQ + QQ - 1 : er - 1; };
  if constexpr (CM) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u >= nz) break;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (v >= ny) break;
        const T* er = row_ptr(u, v);
        T ev[q];
        read_row(er, ev);
#pragma unroll
        for (int j = 0; j < q; ++j) own[j] += ev[j];
        if (c > 0) below += *left_ptr(er);
      }
    }
  } else {
    T ev[2][2][q], evl[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const bool use = u < nz && v < ny;
        const T* er = row_ptr(use ? u : 0, use ? v : 0);
        read_row(er, ev[u][v]);
        evl[u][v] = *(c > 0 ? left_ptr(er) : er);  // (c = 0: an in-row value, weighted out)
      }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const bool use = u < nz && v < ny;
#pragma unroll
        for (int j = 0; j < q; ++j) own[j] += use ? ev[u][v][j] : T(0);
        below += use && c > 0 ? evl[u][v] : T(0);
      }
  }
  const T vyz = T(ny * nz);
#pragma unroll
  for (int j = 0; j < q + 1; ++j) {
    if (j == q && !last) break;
    const int g = g0 + j;
    const int64_t id = row0 + g;
    const bool dir = g == 0 || g == L.nn - 1;
    const T sj = j < q ? (j == 0 && c > 0 ? own[0] + below : own[j < q ? j : 0]) : T(0);
    if (KIND == 0) {
      const T v = dir ? (g == 0 ? xd0 : xd1) : sj;
      out[id] = mode == 2 ? (dir ? T(0) : bv[j] - v) : (mode ? bv[j] - v : v);
    } else if (!dir) {
      const T val = (j == 0 && c > 0) ? vyz * T(2) : vyz;
      out[id] = mode ? omega / val * sj : xv[j] + omega / val * sj;
    } else if (mode) {
      out[id] = T(0);
    }
  }
}

static int gather_lxw(const LevelArgs& L) {
  int l = 0;
  while ((1 << l) < L.n && l < 6) ++l;
  return l;
}
template <int D>
static dim3 gather_grid(const LevelArgs& L, int lxw) {
  const int rows = 256 >> lxw;
  const int64_t nyb = (L.nn + rows - 1) / rows, gy = D == 3 ? nyb * L.nn : nyb, gz = (int64_t)L.N * L.nt * D;
  if (gy > 65535 || gz > 65535) return dim3(0, 0, 0);  // launch fails: invalid configuration
  return dim3((unsigned)((L.n + (1 << lxw) - 1) >> lxw), (unsigned)gy, (unsigned)gz);
}

template <typename T, int KIND>
static hipError_t node_gather(const LevelArgs& L, const T* E, const T* xin, const T* b, T* out, int mode, T omega,
                              hipStream_t s) {
#define STMG_NG(DD, QQ)                                                                                  \
  if (L.d == DD && L.Q == QQ) {                                                                           \
    const int lxw = gather_lxw(L);                                                                      \
    if (KIND == 0 && mode == 2)                                                                           \
      k_node_gather<T, DD, QQ, 0, 2><<<gather_grid<DD>(L, lxw), 256, 0, s>>>(L, E, xin, b, out, omega, lxw); \
    else if (mode)                                                                                        \
      k_node_gather<T, DD, QQ, KIND, 1><<<gather_grid<DD>(L, lxw), 256, 0, s>>>(L, E, xin, b, out, omega, lxw); \
    else                                                                                                  \
      k_node_gather<T, DD, QQ, KIND, 0><<<gather_grid<DD>(L, lxw), 256, 0, s>>>(L, E, xin, b, out, omega, lxw); \
    return hipGetLastError();                                                                             \
  }
  STMG_NG(2, 3) STMG_NG(2, 4) STMG_NG(3, 3) STMG_NG(3, 4)
#undef STMG_NG
  return hipErrorInvalidValue;
}

template <typename T, int D, int Q, int NT>
static hipError_t apply_impl(const LevelArgs& L, const T* geo, const T* tab, const T* x, const T* b, T* y,
                             int mode, T* E, hipStream_t s, bool gather, int nper_req, int variant) {
  constexpr int C = D == 3 ? (Q - 1) * Q * (Q + 1) / 6 : (Q - 1) * Q / 2;
  if (L.C != C || L.nt != NT || L.Q != Q || L.nodes >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  const int64_t ncells = L.Mp / L.C;
  const int64_t nbx = (ncells + 15) / 16;
  // split the subintervals into chunks when there are too few cells to fill the chip
  int64_t nchunk = std::min<int64_t>(L.N, std::max<int64_t>(1, (4096 + 4 * nbx - 1) / (4 * nbx)));
  if (nper_req > 0) nchunk = (L.N + std::min(nper_req, L.N) - 1) / std::min(nper_req, L.N);
  const int nper = (int)((L.N + nchunk - 1) / nchunk);
  nchunk = (L.N + nper - 1) / nper;
  // FP32 3D levels: components inner only when asked (variant 2).  It issues
  // about a quarter fewer instructions but holds 188 registers (2 waves per
  // SIMD against 4), and measured no faster on Q3 levels and slower on Q2
  // levels; FP64 always keeps the components outer (its registers would not fit)
  if constexpr (D == 3 && sizeof(T) == 4) {
    if (variant == 2)
      k_apply<T, D, Q, NT, false, true><<<dim3((unsigned)nbx, (unsigned)nchunk), 256, 0, s>>>(L, geo, tab, x, b, y, E,
                                                                                            mode, nper);
    else
      k_apply<T, D, Q, NT><<<dim3((unsigned)nbx, (unsigned)nchunk), 256, 0, s>>>(L, geo, tab, x, b, y, E, mode, nper);
  } else {
    k_apply<T, D, Q, NT><<<dim3((unsigned)nbx, (unsigned)nchunk), 256, 0, s>>>(L, geo, tab, x, b, y, E, mode, nper);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !gather) return e;
  return node_gather<T, 0>(L, E, x, b, y, mode, T(0), s);
}

template <typename T>
hipError_t launch_apply(const LevelArgs& L, const T* geo, const T* tab, const T* x, const T* b, T* y, int mode,
                        T* E, hipStream_t s, bool gather, int nper, int variant) {
#define STMG_AP(DD, QQ, NN) \
  if (L.d == DD && L.Q == QQ && L.nt == NN)                                                    \
    return apply_impl<T, DD, QQ, NN>(L, geo, tab, x, b, y, mode, E, s, gather, nper, variant);
  STMG_AP(2, 3, 1) STMG_AP(2, 3, 2) STMG_AP(2, 3, 3) STMG_AP(2, 3, 4)
  STMG_AP(2, 4, 1) STMG_AP(2, 4, 2) STMG_AP(2, 4, 3) STMG_AP(2, 4, 4)
  STMG_AP(3, 3, 1) STMG_AP(3, 3, 2) STMG_AP(3, 3, 3) STMG_AP(3, 3, 4)
  STMG_AP(3, 4, 1) STMG_AP(3, 4, 2) STMG_AP(3, 4, 3) STMG_AP(3, 4, 4)
#undef STMG_AP
  return hipErrorInvalidValue;
}

// b_out = f - S_full g - C^1 v0 on free rows and 0 on Dirichlet rows (FP64):
// the right-hand side of the homogeneous slab system for forcing f, Dirichlet
// values g (its entries on free rows are ignored) and the previous slab's end
// value v0 (d x nodes, or null for v0 = 0).
template <int D, int Q, int NT>
static hipError_t lift_impl(const LevelArgs& L, const double* geo, const double* tab, const double* f,
                            const double* g, const double* v0, double* out, double* E, hipStream_t s) {
  constexpr int C = D == 3 ? (Q - 1) * Q * (Q + 1) / 6 : (Q - 1) * Q / 2;
  if (L.C != C || L.nt != NT || L.Q != Q || L.nodes >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  const int64_t nbx = (L.Mp / L.C + 15) / 16;
  // one wave walks every subinterval of its cells: the jump term of the
  // first one reads v0, the others carry it in registers
  k_apply<double, D, Q, NT, true><<<dim3((unsigned)nbx, 1), 256, 0, s>>>(L, geo, tab, g, f, out, E, 1, L.N, v0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return node_gather<double, 0>(L, E, g, f, out, 2, 0.0, s);
}

hipError_t launch_slab_rhs(const LevelArgs& L, const double* geo, const double* tab, const double* f,
                           const double* g, const double* v0, double* out, double* E, hipStream_t s) {
#define STMG_LF(DD, QQ, NN) \
  if (L.d == DD && L.Q == QQ && L.nt == NN) return lift_impl<DD, QQ, NN>(L, geo, tab, f, g, v0, out, E, s);
  STMG_LF(2, 3, 1) STMG_LF(2, 3, 2) STMG_LF(2, 3, 3) STMG_LF(2, 3, 4)
  STMG_LF(2, 4, 1) STMG_LF(2, 4, 2) STMG_LF(2, 4, 3) STMG_LF(2, 4, 4)
  STMG_LF(3, 3, 1) STMG_LF(3, 3, 2) STMG_LF(3, 3, 3) STMG_LF(3, 3, 4)
  STMG_LF(3, 4, 1) STMG_LF(3, 4, 2) STMG_LF(3, 4, 3) STMG_LF(3, 4, 4)
#undef STMG_LF
  return hipErrorInvalidValue;
}

// x = g on every Dirichlet velocity entry of the slab vector (free entries
// and pressure untouched)
__global__ void k_set_dirichlet(LevelArgs L, const double* __restrict__ g, double* __restrict__ x) {
  const int64_t nv = (int64_t)L.N * L.nt * L.d * L.nodes;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nv; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = t % L.nodes, f = t / L.nodes;  // f = (n nt + a) d + comp
    const int64_t comp = f % L.d, na = f / L.d;
    const int gx = (int)(node % L.nn), gy = (int)((node / L.nn) % L.nn), gz = L.d == 3 ? (int)(node / ((int64_t)L.nn * L.nn)) : 1;
    const bool bnd = gx == 0 || gx == L.nn - 1 || gy == 0 || gy == L.nn - 1 || (L.d == 3 && (gz == 0 || gz == L.nn - 1));
    if (bnd) {
      const int64_t id = (na / L.nt) * L.slab + (na % L.nt) * L.Mv + comp * L.nodes + node;
      x[id] = g[id];
    }
  }
}

hipError_t launch_set_dirichlet(const LevelArgs& L, const double* g, double* x, hipStream_t s) {
  k_set_dirichlet<<<2048, 256, 0, s>>>(L, g, x);
  return hipGetLastError();
}

// =====================================================================
// Cell Vanka, Schur-factored local inverse (Eq. (vanka0), (vanka)).
// One work group per spatial cell, all N subintervals at once (the local
// matrix is the same for every subinterval).  Local velocity rows (a, i) per
// component; pressure rows q = (a, l).
//   Z = A_s^{-1} R               (MFMA: mp x mp times mp x (d N), one pass over A_s^{-1})
//   y_p = H^{-1} (D Z - r_p),    y_c = z_c - F_c y_p
//   x_p += omega y_p             (pressure dofs belong to one cell)
//   E   = y_v                    (velocity: summed per node by k_node_gather, KIND 1)
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

template <typename T, int D, int Q, int NT, int NCT>
__global__ __launch_bounds__(256) void k_vanka_mfma(LevelArgs L, const T* __restrict__ Asw,
                                                    const T* __restrict__ Bm, const T* __restrict__ F,
                                                    const T* __restrict__ Hinv, const T* __restrict__ coef,
                                                    const T* __restrict__ r, T* __restrict__ x, T omega,
                                                    T* __restrict__ E, int xzero) {
  constexpr int NL = D == 3 ? Q * Q * Q : Q * Q;
  constexpr int C = D == 3 ? (Q - 1) * Q * (Q + 1) / 6 : (Q - 1) * Q / 2;
  constexpr int M = NT * NL, MP = (M + 15) / 16 * 16, NKB = MP / 16, P = NT * C;
  constexpr int DNP = NCT * 16;
  constexpr int TPW = (NKB + 3) / 4;  // row tiles per wave (4 waves)
  // double-buffer the A_s^{-1} fragments of the next row tile when registers allow
  constexpr bool DB = TPW > 1 && NKB * 4 * (int)sizeof(T) <= 192;
  typedef typename mfma_vec<T>::v4 v4;
  const int N = L.N, lgN = N == 1 ? 0 : (N == 2 ? 1 : (N == 4 ? 2 : 3)), DN = D * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // Z rows are padded by one value (ZS): consecutive rows fall on consecutive banks
  constexpr int ZS = DNP + 1;
  constexpr int P4 = (P + 3) / 4 * 4;      // row length of F and H^{-1} (vanka_row_pad), and of YP
  // the Schur sums over (comp, node) are split KS ways so that P N KS items fill the work group
  constexpr int KS = P * 8 >= 256 ? 1 : (P * 8 >= 128 ? 2 : 4);
  T* RZ = reinterpret_cast<T*>(smem_raw);  // R (B-operand order), then Z (row-major MP x ZS)
  T* YP = RZ + MP * ZS;                    // y_p as [n][q] (rows of P4, 16-byte aligned)
  T* sB = YP + 8 * P4;                     // B of this cell, [comp][i][l] (l fastest: no bank conflicts)
  T* Rp = sB + C * D * NL;                 // pressure residual [q][n]
  T* S = Rp + P * 8;                       // Schur right-hand side [q][n]
  T* Sp = S + P * 8;                       // its KS partial sums [k][q][n]
  T* sc = Sp + KS * P * 8;
  const int64_t cell = xcd_remap(blockIdx.x, gridDim.x);
  int cc[3];
  cell_coords(L, cell, cc);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;

  // ---- A_s^{-1} fragments of this wave's first row tile: issued first, so
  // that their latency overlaps the residual gather
  const T* A = Asw + cell * (int64_t)MP * MP;
  T fa[2][NKB][4];
  auto load_tile = [&](int t, T (&f)[NKB][4]) {
    const T* At = A + (int64_t)t * NKB * 256 + lane * 4;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
      for (int j = 0; j < 4; ++j) f[kb][j] = At[kb * 256 + j];
  };

  // ---- R in B-operand order, B and the pressure residual.  R is read one
  // x-row of a cell (Q consecutive nodes, one vector load) of every temporal
  // dof per item: items (n, comp, row), n fastest (so that the 16-byte LDS
  // stores of a wave spread over all banks), the index work shared by the
  // temporal dofs; Dirichlet entries are zeroed in registers.  Padding
  // entries of R (K >= M or column >= d N) are zeroed separately.  Loads
  // complete in issue order, so the loads this phase waits for are issued
  // first, then the A_s^{-1} fragments of the first row tile (consumed only
  // after the barrier).
  {
    constexpr int ROWS = NL / Q;                      // x-rows of a cell
    constexpr int IMAX = (ROWS * D * 8 + 255) / 256;  // items per thread (N <= 8)
    constexpr int PB = (C * D * NL + 255) / 256;
    const int nitems = ROWS * DN;
    const T* Bc = Bm + cell * (int64_t)C * D * NL;
    T rv[IMAX][NT][Q], bv[PB];
    bool rok[IMAX];
    // unconditional loads from clamped (in-bounds) addresses, selected later:
    // the wait counts before the first LDS store then stay exact
#pragma unroll
    for (int e = 0; e < IMAX; ++e) {
      const int it = min(tid + 256 * e, nitems - 1);
      const int n = it & (N - 1), rest = it >> lgN, comp = rest % D, row = rest / D;
      const int iy = row % Q, iz = row / Q;
      const int gy = cc[1] * (Q - 1) + iy, gz = D == 3 ? cc[2] * (Q - 1) + iz : 1;
      rok[e] = tid + 256 * e < nitems && gy > 0 && gy < L.nn - 1 && gz > 0 && (D == 2 || gz < L.nn - 1);
      const int64_t g = (int64_t)cc[0] * (Q - 1) + (int64_t)L.nn * (gy + (D == 3 ? (int64_t)L.nn * gz : 0));
      const T* rp = r + vidx(L, n, 0, comp, g);
#pragma unroll
      for (int a = 0; a < NT; ++a) __builtin_memcpy(rv[e][a], rp + (int64_t)a * L.Mv, sizeof(T) * Q);
    }
#pragma unroll
    for (int e = 0; e < PB; ++e) bv[e] = Bc[min(tid + 256 * e, C * D * NL - 1)];
    constexpr int PR = (P * 8 + 255) / 256;
    T pv[PR];
#pragma unroll
    for (int e = 0; e < PR; ++e) {
      const int t = min(tid + 256 * e, P * N - 1), q = t >> lgN, n = t & (N - 1);
      pv[e] = r[pidx(L, n, q / C, cell, q % C)];
    }
    const T cv = coef[min(tid, NT - 1)];
    load_tile(min(wave, NKB - 1), fa[0]);
    // padding entries (K >= M or column >= d N): only the last row tile and
    // the last column tile hold any; one entry of a tile per thread
    {
      const int l64 = tid >> 2, sl = tid & 3;
      for (int tile = 0; tile < NCT * NKB; ++tile) {
        const int kb = tile % NKB, ct = tile / NKB;
        if (!((kb == NKB - 1 && M < MP) || (ct == NCT - 1 && DN < DNP))) continue;  // (uniform)
        const int K = kb * 16 + 4 * (l64 >> 4) + sl, col = ct * 16 + (l64 & 15);
        if (K >= M || col >= DN) RZ[tile * 256 + tid] = T(0);
      }
    }
#pragma unroll
    for (int e = 0; e < IMAX; ++e) {
      const int it = tid + 256 * e;
      if (it < nitems) {
        const int n = it & (N - 1), rest = it >> lgN, comp = rest % D, row = rest / D, col = comp * N + n;
        const int ct = col / 16, jj = col % 16;
        // Dirichlet rows, and Dirichlet nodes at the ends of the row (x = 0, x = 1)
        bool zero[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j)
          zero[j] = !rok[e] || (j == 0 && cc[0] == 0) || (j == Q - 1 && cc[0] == L.n - 1);
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int j = 0; j < Q; ++j) {
            const int K = a * NL + row * Q + j, kb = K / 16, rem = K % 16;
            RZ[((ct * NKB + kb) * 64 + jj + 16 * (rem / 4)) * 4 + (rem % 4)] = zero[j] ? T(0) : rv[e][a][j];
          }
      }
    }
#pragma unroll
    for (int e = 0; e < PB; ++e) {
      const int idx = tid + 256 * e;  // global order [l][comp][i]
      if (idx < C * D * NL) {
        const int l = idx / (D * NL), ci = idx - l * (D * NL);
        sB[ci * C + l] = bv[e];
      }
    }
#pragma unroll
    for (int e = 0; e < PR; ++e)
      if (tid + 256 * e < P * N) Rp[tid + 256 * e] = pv[e];
    if (tid < NT) sc[tid] = cv;
  }
  __syncthreads();

  // ---- Z = A_s^{-1} R on the matrix cores, one 16-row tile at a time
  v4 acc[TPW][NCT];
#pragma unroll
  for (int it = 0; it < TPW; ++it) {
    const int t = wave + it * 4;
    T (&cur)[NKB][4] = fa[DB ? (it & 1) : 0];
    // tile loads are unconditional (clamped tile index): a load under a branch
    // makes the compiler wait for it even where it was not issued, and the
    // MFMAs of this tile would wait for the next tile's loads
    if (!DB && it > 0) load_tile(min(t, NKB - 1), cur);
    if (DB && it + 1 < TPW) load_tile(min(t + 4, NKB - 1), fa[(it + 1) & 1]);
    if (t < NKB) {
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[it][ct] = v4{0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const T* bp = RZ + ((ct * NKB + kb) * 64 + lane) * 4;
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[it][ct] = mfma_vec<T>::mma(cur[kb][j], bp[j], acc[it][ct]);
        }
    }
  }
  __syncthreads();  // every wave is done reading R
#pragma unroll
  for (int it = 0; it < TPW; ++it) {
    const int t = wave + it * 4;
    if (t < NKB)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          RZ[(t * 16 + mfma_vec<T>::row(lane, v)) * ZS + ct * 16 + lane % 16] = acc[it][ct][v];
  }
  // F and H^{-1} rows of this thread (16-byte loads), issued now (the A
  // fragments are dead) so that their latency overlaps the Schur complement
  constexpr int RPT = (D * M + 255) / 256;  // velocity rows per thread
  constexpr int HPT = (P * 8 + 255) / 256;  // (pp, n) items per thread, N <= 8
  const T* Fc = F + cell * (int64_t)D * M * P4;
  const T* H = Hinv + cell * (int64_t)P * P4;
  T fv[RPT][P], hv[HPT][P], xp[HPT];
  // (unconditional loads from clamped addresses: exact wait counts)
#pragma unroll
  for (int j = 0; j < HPT; ++j) {
    const int t = min(tid + 256 * j, P * N - 1), pp = t >> lgN, n = t & (N - 1);
    {
      T hrow[P4];
      __builtin_memcpy(hrow, __builtin_assume_aligned(H + pp * P4, 16), sizeof(T) * P4);
#pragma unroll
      for (int q = 0; q < P; ++q) hv[j][q] = hrow[q];
    }
    xp[j] = x[pidx(L, n, pp / C, cell, pp % C)];
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int row2 = min(tid + 256 * j, D * M - 1);
    {
      T frow[P4];
      __builtin_memcpy(frow, __builtin_assume_aligned(Fc + (int64_t)row2 * P4, 16), sizeof(T) * P4);
#pragma unroll
      for (int q = 0; q < P; ++q) fv[j][q] = frow[q];
    }
  }
  __syncthreads();
  const T* Z = RZ;

  // ---- pressure Schur complement: S = -c_a B Z - r_p, y_p = H^{-1} S.  The
  // sums over the local nodes are split KS ways (item t = (q n) KS + k), the
  // partial sums added in a fixed order after a barrier.
  constexpr int ISPL = (NL + KS - 1) / KS;
  for (int t = tid; t < P * N * KS; t += 256) {
    const int k = t % KS, it = t / KS, q = it >> lgN, n = it & (N - 1), a = q / C, l = q % C;
    T s = 0;
#pragma unroll
    for (int comp = 0; comp < D; ++comp)
#pragma unroll
      for (int ii = 0; ii < ISPL; ++ii) {
        const int i = k * ISPL + ii;
        if (i < NL) s += sB[(comp * NL + i) * C + l] * Z[(a * NL + i) * ZS + comp * N + n];
      }
    Sp[k * P * 8 + it] = s;
  }
  __syncthreads();
  for (int t = tid; t < P * N; t += 256) {
    T s = 0;
#pragma unroll
    for (int k = 0; k < KS; ++k) s += Sp[k * P * 8 + t];
    S[t] = -sc[(t >> lgN) / C] * s - Rp[t];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < HPT; ++j) {
    const int t = tid + 256 * j;
    if (t < P * N) {
      const int pp = t >> lgN, n = t & (N - 1);
      T s = 0;
#pragma unroll
      for (int q = 0; q < P; ++q) s += hv[j][q] * S[q * N + n];
      YP[n * P4 + pp] = s;
      x[pidx(L, n, pp / C, cell, pp % C)] = (xzero ? T(0) : xp[j]) + omega * s;  // xzero: x starts at 0
    }
  }
  __syncthreads();

  // ---- velocity: y = z - F y_p into the cell-local scratch E (cell-major:
  // the work group writes whole cache lines; e_index, field (n NT + a) D + comp)
  const int64_t nstride = (int64_t)NT * D * n_cells(L) * NL;  // between fields (n, a) and (n + 1, a)
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int row2 = tid + 256 * j;
    if (row2 >= D * M) break;
    const int comp = row2 / M, row = row2 % M, a = row / NL, i = row % NL;
    const T(&f)[P] = fv[j];
    T* ep = E + e_index(L, a * D + comp, cell, i);
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      if (n >= N) break;
      T yp[P4];
      __builtin_memcpy(yp, __builtin_assume_aligned(YP + n * P4, 16), sizeof(yp));
      T v = Z[row * ZS + comp * N + n];
#pragma unroll
      for (int q = 0; q < P; ++q) v = fma(-f[q], yp[q], v);
      *ep = v;
      ep += nstride;
    }
  }
}

template <typename T>
static hipError_t vanka_gather(const LevelArgs& L, const T* E, T* x, T omega, hipStream_t s, bool xzero = false) {
  return node_gather<T, 1>(L, E, nullptr, nullptr, x, xzero ? 1 : 0, omega, s);
}

template <typename T, int D, int Q, int NT>
static hipError_t vanka_fact_impl(const LevelArgs& L, const T* Asw, const T* Bm, const T* F, const T* Hinv,
                                  const T* coef, const T* r, T* x, T omega, T* E, hipStream_t s, bool gather,
                                  bool xzero) {
  constexpr int NL = D == 3 ? Q * Q * Q : Q * Q;
  constexpr int C = D == 3 ? (Q - 1) * Q * (Q + 1) / 6 : (Q - 1) * Q / 2;
  constexpr int M = NT * NL, MP = (M + 15) / 16 * 16, P = NT * C;
  if (L.C != C || L.nloc != NL || L.nt != NT || L.N < 1 || L.N > 8 || (L.N & (L.N - 1))) return hipErrorInvalidValue;
  if (MP / 16 > 16) return hipErrorInvalidValue;  // at most 4 row tiles per wave
  const int64_t ncells = L.Mp / L.C;
  const int DN = D * L.N;
  constexpr int P4 = (P + 3) / 4 * 4, KS = P * 8 >= 256 ? 1 : (P * 8 >= 128 ? 2 : 4);
  auto shm = [&](int dnp) {
    return sizeof(T) * ((size_t)MP * (dnp + 1) + 8 * (size_t)P4 + (size_t)C * D * NL + (2 + KS) * (size_t)P * 8 + 8);
  };
  auto run = [&](auto kern, size_t bytes) -> hipError_t {
    if (bytes > 65536) {  // beyond the default dynamic LDS limit
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e != hipSuccess) return e;
    }
    kern<<<(unsigned)ncells, 256, bytes, s>>>(L, Asw, Bm, F, Hinv, coef, r, x, omega, E, xzero ? 1 : 0);
    return hipSuccess;
  };
  hipError_t e;
  if (DN <= 16) {
    e = run(k_vanka_mfma<T, D, Q, NT, 1>, shm(16));
  } else if (DN <= 32) {
    e = run(k_vanka_mfma<T, D, Q, NT, 2>, shm(32));
  } else {
    return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (!gather) return hipGetLastError();
  return vanka_gather<T>(L, E, x, omega, s, xzero);
}

template <typename T>
hipError_t launch_vanka_gather_only(const LevelArgs& L, const T* E, T* x, T omega, hipStream_t s, bool xzero) {
  return vanka_gather<T>(L, E, x, omega, s, xzero);
}

template <typename T>
hipError_t launch_vanka_factored(const LevelArgs& L, const T* Asw, const T* Bm, const T* F, const T* Hinv,
                                 const T* coef, const T* r, T* x, T omega, T* E, hipStream_t s, bool gather,
                                 bool xzero) {
#define STMG_VF(DD, QQ, KK)                                                                                   \
  if (L.d == DD && L.Q == QQ && L.nt == KK)                                                                   \
    return vanka_fact_impl<T, DD, QQ, KK>(L, Asw, Bm, F, Hinv, coef, r, x, omega, E, s, gather, xzero);
  STMG_VF(2, 3, 1) STMG_VF(2, 3, 2) STMG_VF(2, 3, 3) STMG_VF(2, 3, 4)
  STMG_VF(2, 4, 1) STMG_VF(2, 4, 2) STMG_VF(2, 4, 3) STMG_VF(2, 4, 4)
  STMG_VF(3, 3, 1) STMG_VF(3, 3, 2) STMG_VF(3, 3, 3) STMG_VF(3, 3, 4)
  STMG_VF(3, 4, 1) STMG_VF(3, 4, 2) STMG_VF(3, 4, 3) STMG_VF(3, 4, 4)
#undef STMG_VF
  return hipErrorInvalidValue;
}

// =====================================================================
// Cell Vanka with the temporally decoupled factors (one spatial Stokes block
// per eigenvalue of diag(c)^{-1} K; host.hpp, TemporalEigen).  One work group
// per spatial cell, all N subintervals and d components at once:
//   R~_j = sum_a T_ja R_a                 (velocity and pressure residuals)
//   Z_j  = Ainv_j R~_j                    (matrix cores; a complex block as
//                                          the real operands Re / Im Ainv_j,
//                                          each symmetric and stored as its
//                                          upper 16 x 16 tiles)
//   p~_j = Hinv_j (-B Z_j - R~p_j),  u~_j = Z_j - F_j p~_j
//   x_p[a] += omega sum_j Re(Wt_aj p~_j),  E[a] = sum_j Re(Wt_aj u~_j)
// Columns of R~ and Z: comp N + n, padded to DNP = 16 NCT; real parts, then
// imaginary parts (a real block's are zero and never read).  Block j's Ainv
// tiles are streamed once from HBM; a complex block needs both Re and Im.
// =====================================================================
// DIAG: the diagonal Vanka's blocks lambda_j diag(M) + diag(A): Aw holds
// their inverses as nloc complex values per block (re, im), Z_j is formed
// elementwise while the residual is staged, and F_j = -Dinv_j B^T is formed
// from B (Ft is not read).
// FP32 with at most two temporal dofs: at most 96 registers (5 waves per
// SIMD, as many as the shared memory allows), measured 3% faster than the
// unconstrained 104 on the Q3 x DG(1) level of 32^3 cells; FP64 and more
// temporal dofs keep their registers (they would spill).
template <typename T, int D, int Q, int NT, int NCT, bool DIAG = false>
__global__ __launch_bounds__(256, sizeof(T) == 4 && NT <= 2 ? 5 : 1) void k_vanka_tdec(LevelArgs L, const T* __restrict__ Aw,
                                                    const T* __restrict__ Bm, const T* __restrict__ Ft,
                                                    const T* __restrict__ Ht, const T* __restrict__ tw,
                                                    const T* __restrict__ r, T* __restrict__ x, T omega,
                                                    T* __restrict__ E, int xzero) {
  constexpr int NL = D == 3 ? Q * Q * Q : Q * Q;
  constexpr int C = D == 3 ? (Q - 1) * Q * (Q + 1) / 6 : (Q - 1) * Q / 2;
  constexpr int MP = (NL + 15) / 16 * 16, NKB = MP / 16;
  constexpr int J = (NT + 1) / 2, NR = NT % 2;  // blocks; block 0 is real iff NT is odd
  constexpr int DNP = NCT * 16, NCOL = 2 * DNP, ZS = NCOL + 1;
  constexpr int RT = J * NKB;                   // row tiles (16 rows of one block)
  constexpr int NTL = NKB * (NKB + 1) / 2;      // stored (upper) tiles of one real block
  constexpr int CSPL = RT >= 4 ? 1 : 4 / RT;    // waves that share a row tile split its column tiles
  constexpr int TPW = (RT + 3) / 4;             // row tiles per wave
  constexpr int R4 = (2 * C + 3) / 4 * 4;       // vanka_tdec_row(C)
  typedef typename mfma_vec<T>::v4 v4;
  const int N = L.N, lgN = N == 1 ? 0 : (N == 2 ? 1 : (N == 4 ? 2 : 3)), DN = D * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* RZ = reinterpret_cast<T*>(smem_raw);  // R~ in B-operand order, then Z as [j][row][ZS]
  // complex vectors of C values per (j, n), as (re, im) pairs in rows of R4
  // (16-byte aligned): one row is read with a few wide loads
  T* Sc = RZ + J * MP * ZS;                // Schur right-hand side [j][n][l]
  T* Pc = Sc + J * 8 * R4;                 // p~ [j][n][l]
  T* sB = Pc + J * 8 * R4;                 // B of this cell, [comp][i][l]
  T* Rp = sB + C * D * NL;                 // pressure residual as read, [a C + l][n]
  T* Sp = Rp + NT * C * 8;                 // per wave: partial (B Z_j)^T tiles [wave][j][16][17]
  const T* tT = tw;                  // T[j][a] (re, im)
  const T* tW = tw + 2 * J * NT;     // Wt[a][j] (re, im)
  const int64_t cell = xcd_remap(blockIdx.x, gridDim.x);
  int cc[3];
  cell_coords(L, cell, cc);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  auto ridx = [](int j, int part, int ct, int kb, int ln, int slot) {
    return ((((j * 2 + part) * NCT + ct) * NKB + kb) * 64 + ln) * 4 + slot;
  };

  // ---- Ainv fragments of this wave's first row tile (issued right after
  // the residual loads, consumed after the barrier).  Tile (lt, kb) with
  // kb < lt is read from its mirror (kb, lt) and transposed before use.
  const T* A = Aw + cell * (int64_t)(DIAG ? 2 * J * NL : NT * NTL * 256);
  T fx[NKB][4], fy[NKB][4];
  auto load_tile = [&](int t) {
    if constexpr (DIAG) return;
    const int j = t / NKB, lt = t % NKB;
    const T* X = A + (int64_t)(j < NR ? j : 2 * j - NR) * NTL * 256 + lane * 4;
    const T* Y = j < NR ? X : X + NTL * 256;  // (a real block reads its Re tile twice; unused)
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      const int I = min(lt, kb), K = max(lt, kb), up = I * NKB - I * (I - 1) / 2 + (K - I);
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        fx[kb][sl] = X[up * 256 + sl];
        fy[kb][sl] = Y[up * 256 + sl];
      }
    }
  };
  const int t_first = CSPL > 1 ? wave % RT : min(wave, RT - 1);

  // ---- residual rows to the temporal eigenbasis, in B-operand order.  Items
  // (n, comp, x-row), n fastest; each reads the x-row (Q nodes) of every
  // temporal dof, zeroes Dirichlet entries and writes R~_j of its Q nodes.
  {
    constexpr int ROWS = NL / Q;
    constexpr int IMAX = (ROWS * D * 8 + 255) / 256;  // N <= 8
    constexpr int PB = (C * D * NL + 255) / 256;
    constexpr int PR = (NT * C * 8 + 255) / 256;
    const int nitems = ROWS * DN;
    const T* Bc = Bm + cell * (int64_t)C * D * NL;
    T rv[IMAX][NT][Q], bv[PB], pv[PR];
    bool rok[IMAX];
    // unconditional loads from clamped (in-bounds) addresses
#pragma unroll
    for (int e = 0; e < IMAX; ++e) {
      const int it = min(tid + 256 * e, nitems - 1);
      const int n = it & (N - 1), rest = it >> lgN, comp = rest % D, row = rest / D;
      const int iy = row % Q, iz = row / Q;
      const int gy = cc[1] * (Q - 1) + iy, gz = D == 3 ? cc[2] * (Q - 1) + iz : 1;
      rok[e] = tid + 256 * e < nitems && gy > 0 && gy < L.nn - 1 && gz > 0 && (D == 2 || gz < L.nn - 1);
      const int64_t g = (int64_t)cc[0] * (Q - 1) + (int64_t)L.nn * (gy + (D == 3 ? (int64_t)L.nn * gz : 0));
#pragma unroll
      for (int a = 0; a < NT; ++a) __builtin_memcpy(rv[e][a], r + vidx(L, n, a, comp, g), sizeof(T) * Q);
    }
#pragma unroll
    for (int e = 0; e < PB; ++e) bv[e] = Bc[min(tid + 256 * e, C * D * NL - 1)];
#pragma unroll
    for (int e = 0; e < PR; ++e) {
      const int t = min(tid + 256 * e, NT * C * N - 1), q = t >> lgN, n = t & (N - 1);
      pv[e] = r[pidx(L, n, q / C, cell, q % C)];
    }
    load_tile(t_first);
    // padding entries (rows >= NL or columns >= d N): only the last row tile
    // and the last column tile hold any; one entry of a tile per thread.
    // DIAG writes Z directly: its rows NL..MP-1 are zeroed instead.
    if constexpr (DIAG) {
      for (int idx = tid; idx < J * (MP - NL) * NCOL; idx += 256) {
        const int j = idx / ((MP - NL) * NCOL), rest = idx % ((MP - NL) * NCOL);
        RZ[(j * MP + NL + rest / NCOL) * ZS + rest % NCOL] = T(0);
      }
    } else {
      const int l64 = tid >> 2, sl = tid & 3;
      for (int tile = 0; tile < J * 2 * NCT * NKB; ++tile) {
        const int kb = tile % NKB, ct = (tile / NKB) % NCT;
        if (!((kb == NKB - 1 && NL < MP) || (ct == NCT - 1 && DN < DNP))) continue;  // (uniform)
        const int K = kb * 16 + 4 * (l64 >> 4) + sl, col = ct * 16 + (l64 & 15);
        if (K >= NL || col >= DN) RZ[tile * 256 + tid] = T(0);
      }
    }
#pragma unroll
    for (int e = 0; e < IMAX; ++e) {
      const int it = tid + 256 * e;
      if (it < nitems) {
        const int n = it & (N - 1), rest = it >> lgN, comp = rest % D, row = rest / D;
        const int col = comp * N + n, ct = col / 16, jj = col % 16, K0 = row * Q;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int q = 0; q < Q; ++q)
            if (!rok[e] || (q == 0 && cc[0] == 0) || (q == Q - 1 && cc[0] == L.n - 1)) rv[e][a][q] = T(0);
#pragma unroll
        for (int j = 0; j < J; ++j) {
          T tr[NT], ti[NT];
#pragma unroll
          for (int a = 0; a < NT; ++a) {
            tr[a] = tT[(j * NT + a) * 2];
            ti[a] = tT[(j * NT + a) * 2 + 1];
          }
          T sr[Q], si[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            sr[q] = 0;
            si[q] = 0;
#pragma unroll
            for (int a = 0; a < NT; ++a) {
              sr[q] += tr[a] * rv[e][a][q];
              si[q] += ti[a] * rv[e][a][q];
            }
          }
          if constexpr (DIAG) {
            // Z_j = Dinv_j R~_j, written in Z's row-major layout
            const T* dv = A + (j * NL + K0) * 2;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
              const T dr = dv[2 * q], di = dv[2 * q + 1];
              T* zz = RZ + (j * MP + K0 + q) * ZS + col;
              zz[0] = dr * sr[q] - di * si[q];
              zz[DNP] = dr * si[q] + di * sr[q];
            }
          } else if constexpr (Q == 4) {
            // the row's 4 nodes are the 4 slots of one lane: one wide store
            const int ln = jj + 16 * (row % 4);
            __builtin_memcpy(RZ + ridx(j, 0, ct, row / 4, ln, 0), sr, sizeof(sr));
            if (j >= NR) __builtin_memcpy(RZ + ridx(j, 1, ct, row / 4, ln, 0), si, sizeof(si));
          } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
              const int K = K0 + q, kb = K / 16, rem = K % 16, ln = jj + 16 * (rem / 4);
              RZ[ridx(j, 0, ct, kb, ln, rem % 4)] = sr[q];
              if (j >= NR) RZ[ridx(j, 1, ct, kb, ln, rem % 4)] = si[q];
            }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < PB; ++e) {
      const int idx = tid + 256 * e;  // global order [l][comp][i]
      if (idx < C * D * NL) {
        const int l = idx / (D * NL), ci = idx - l * (D * NL);
        sB[ci * C + l] = bv[e];
      }
    }
#pragma unroll
    for (int e = 0; e < PR; ++e)
      if (tid + 256 * e < NT * C * N) Rp[tid + 256 * e] = pv[e];
  }
  __syncthreads();

  // ---- Z_j = Ainv_j R~_j on the matrix cores, one 16-row tile at a time:
  // Re Z = X Re R~ - Y Im R~, Im Z = X Im R~ + Y Re R~ (X, Y: Re, Im Ainv_j)
  v4 accR[TPW][NCT], accI[TPW][NCT];
  const int cpart = CSPL > 1 ? wave / RT : 0;
#pragma unroll
  for (int it = 0; it < (DIAG ? 0 : TPW); ++it) {
    const int t = CSPL > 1 ? t_first : wave + 4 * it;
    if (it > 0) load_tile(min(t, RT - 1));  // unconditional (clamped): exact wait counts
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      accR[it][ct] = v4{0, 0, 0, 0};
      accI[it][ct] = v4{0, 0, 0, 0};
    }
    const bool active = t < RT && (CSPL == 1 || wave < RT * CSPL);
    if (active) {
      const int j = t / NKB, lt = t % NKB;
#pragma unroll
      for (int kb = 0; kb < NKB - 1; ++kb)
        if (kb < lt) {  // (wave-uniform) a tile below the diagonal
          tile_transpose16<T>(fx[kb], lane);
          if (j >= NR) tile_transpose16<T>(fy[kb], lane);
        }
      if (j >= NR) {
        T ny[NKB][4];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
          for (int sl = 0; sl < 4; ++sl) ny[kb][sl] = -fy[kb][sl];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
          for (int sl = 0; sl < 4; ++sl)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
              if (CSPL > 1 && ct % CSPL != cpart) continue;
              const T bR = RZ[ridx(j, 0, ct, kb, lane, sl)], bI = RZ[ridx(j, 1, ct, kb, lane, sl)];
              accR[it][ct] = mfma_vec<T>::mma(fx[kb][sl], bR, accR[it][ct]);
              accI[it][ct] = mfma_vec<T>::mma(fx[kb][sl], bI, accI[it][ct]);
              accR[it][ct] = mfma_vec<T>::mma(ny[kb][sl], bI, accR[it][ct]);
              accI[it][ct] = mfma_vec<T>::mma(fy[kb][sl], bR, accI[it][ct]);
            }
      } else {
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
          for (int sl = 0; sl < 4; ++sl)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
              if (CSPL > 1 && ct % CSPL != cpart) continue;
              accR[it][ct] = mfma_vec<T>::mma(fx[kb][sl], RZ[ridx(j, 0, ct, kb, lane, sl)], accR[it][ct]);
            }
      }
    }
  }
  __syncthreads();  // every wave is done reading R~
#pragma unroll
  for (int it = 0; it < (DIAG ? 0 : TPW); ++it) {
    const int t = CSPL > 1 ? t_first : wave + 4 * it;
    const bool active = t < RT && (CSPL == 1 || wave < RT * CSPL);
    if (active) {
      const int j = t / NKB, lt = t % NKB;
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        if (CSPL > 1 && ct % CSPL != cpart) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T* zr = RZ + (j * MP + lt * 16 + mfma_vec<T>::row(lane, v)) * ZS + ct * 16 + lane % 16;
          zr[0] = accR[it][ct][v];
          zr[DNP] = accI[it][ct][v];  // zero for a real block
        }
      }
    }
  }
  // F and Hinv rows of this thread and the old pressure values, issued now
  // (the Ainv fragments are dead) so that their latency overlaps the Schur
  // complement
  constexpr int RPT = (D * NL + 255) / 256;       // velocity rows (comp, i) per thread
  constexpr int HPT = (J * C * 8 + 255) / 256;    // (j, l', n) items per thread, N <= 8
  constexpr int XPT = (NT * C * 8 + 255) / 256;   // (a, l, n) items per thread
  const T* Fc = Ft + cell * (int64_t)J * D * NL * R4;
  const T* Hc = Ht + cell * (int64_t)J * C * R4;
  T fv[RPT][J][2 * C], hv[HPT][2 * C], xp[XPT];
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int t = min(tid + 256 * h, J * C * N - 1), pp = t >> lgN;
    T hrow[R4];
    __builtin_memcpy(hrow, __builtin_assume_aligned(Hc + pp * R4, 16), sizeof(T) * R4);
#pragma unroll
    for (int q = 0; q < 2 * C; ++q) hv[h][q] = hrow[q];
  }
#pragma unroll
  for (int e = 0; e < XPT; ++e) {
    const int t = min(tid + 256 * e, NT * C * N - 1), q = t >> lgN, n = t & (N - 1);
    xp[e] = x[pidx(L, n, q / C, cell, q % C)];
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int row2 = min(tid + 256 * k, D * NL - 1);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if constexpr (DIAG) {  // F_j[comp][i][l] = -Dinv_j[i] B[l][comp][i] (B in LDS since the first barrier)
        const int i = row2 % NL;
        const T dr = A[(j * NL + i) * 2], di = A[(j * NL + i) * 2 + 1];
#pragma unroll
        for (int l = 0; l < C; ++l) {
          const T bb = sB[row2 * C + l];
          fv[k][j][2 * l] = -dr * bb;
          fv[k][j][2 * l + 1] = -di * bb;
        }
      } else {
        T frow[R4];
        __builtin_memcpy(frow, __builtin_assume_aligned(Fc + ((int64_t)j * D * NL + row2) * R4, 16), sizeof(T) * R4);
#pragma unroll
        for (int q = 0; q < 2 * C; ++q) fv[k][j][q] = frow[q];
      }
    }
  }
  __syncthreads();
  const T* Z = RZ;

  // ---- Schur complement right-hand side S_j = -B Z_j - R~p_j.  (B Z_j)^T on
  // the matrix cores: rows m = 8 part + n (real / imaginary part of Z_j's
  // column (comp, n)), columns l, k = comp MP + i, the k-blocks split over the
  // waves; rows i >= NL of Z_j are zero (so are Ainv_j's padding rows), and
  // rows n >= N and columns l >= C are not used (their operands are clamped)
  {
    constexpr int KB = D * MP / 16, KPW = (KB + 3) / 4;
    const int m = lane % 16, part = m / 8, nz = min(m % 8, N - 1), lc = min(lane % 16, C - 1);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      v4 sacc = v4{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < KPW; ++kk) {
        const int kb = wave + 4 * kk;
        if (kb < KB) {
#pragma unroll
          for (int sl = 0; sl < 4; ++sl) {
            const int k = kb * 16 + 4 * (lane / 16) + sl, comp = k / MP, i = k % MP;
            const T av = Z[(j * MP + i) * ZS + part * DNP + comp * N + nz];
            const T bvv = sB[(comp * NL + min(i, NL - 1)) * C + lc];
            sacc = mfma_vec<T>::mma(av, bvv, sacc);
          }
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Sp[((wave * J + j) * 16 + mfma_vec<T>::row(lane, v)) * 17 + lane % 16] = sacc[v];
    }
  }
  __syncthreads();
  for (int t = tid; t < J * C * N; t += 256) {
    const int n = t & (N - 1), q = t >> lgN, j = q / C, l = q % C;
    T sr = 0, si = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sr += Sp[((w * J + j) * 16 + n) * 17 + l];
      si += Sp[((w * J + j) * 16 + 8 + n) * 17 + l];
    }
    T pr = 0, pi = 0;
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const T v = Rp[(a * C + l) * N + n];
      pr += tT[(j * NT + a) * 2] * v;
      pi += tT[(j * NT + a) * 2 + 1] * v;
    }
    Sc[(j * N + n) * R4 + 2 * l] = -sr - pr;
    Sc[(j * N + n) * R4 + 2 * l + 1] = -si - pi;
  }
  __syncthreads();
  // ---- p~_j = Hinv_j S_j
#pragma unroll
  for (int h = 0; h < HPT; ++h) {
    const int t = tid + 256 * h;
    if (t < J * C * N) {
      const int pp = t >> lgN, n = t & (N - 1), j = pp / C;
      T sv[R4];
      __builtin_memcpy(sv, __builtin_assume_aligned(Sc + (j * N + n) * R4, 16), sizeof(sv));
      T pr = 0, pi = 0;
#pragma unroll
      for (int l = 0; l < C; ++l) {
        const T hr = hv[h][2 * l], hi = hv[h][2 * l + 1], sr = sv[2 * l], si = sv[2 * l + 1];
        pr = fma(hr, sr, fma(-hi, si, pr));
        pi = fma(hr, si, fma(hi, sr, pi));
      }
      Pc[(j * N + n) * R4 + 2 * (pp - j * C)] = pr;
      Pc[(j * N + n) * R4 + 2 * (pp - j * C) + 1] = pi;
    }
  }
  __syncthreads();
  // ---- pressure: x_p[a] += omega sum_j Re(Wt_aj p~_j) (cell-owned dofs)
#pragma unroll
  for (int e = 0; e < XPT; ++e) {
    const int t = tid + 256 * e;
    if (t < NT * C * N) {
      const int q = t >> lgN, n = t & (N - 1), a = q / C, l = q % C;
      T v = 0;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const T* pc = Pc + (j * N + n) * R4 + 2 * l;
        v = fma(tW[(a * J + j) * 2], pc[0], fma(-tW[(a * J + j) * 2 + 1], pc[1], v));
      }
      x[pidx(L, n, a, cell, l)] = (xzero ? T(0) : xp[e]) + omega * v;
    }
  }
  // ---- velocity: u~_j = Z_j - F_j p~_j, E[a] = sum_j Re(Wt_aj u~_j) (cell-major,
  // e_index: field (n NT + a) D + comp)
  const int64_t fstride = (int64_t)D * n_cells(L) * NL;  // between fields (n, a) and (n, a + 1)
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int row2 = tid + 256 * k;
    if (row2 >= D * NL) break;
    const int comp = row2 / NL, i = row2 % NL;
    T* ep = E + e_index(L, comp, cell, i);
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      if (n >= N) break;
      T ur[J], ui[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const T* zz = Z + (j * MP + i) * ZS + comp * N + n;
        T pv2[R4];
        __builtin_memcpy(pv2, __builtin_assume_aligned(Pc + (j * N + n) * R4, 16), sizeof(pv2));
        T vr = zz[0], vi = zz[DNP];
#pragma unroll
        for (int l = 0; l < C; ++l) {
          const T fr = fv[k][j][2 * l], fi = fv[k][j][2 * l + 1], pr = pv2[2 * l], pi = pv2[2 * l + 1];
          vr = fma(-fr, pr, fma(fi, pi, vr));
          vi = fma(-fr, pi, fma(-fi, pr, vi));
        }
        ur[j] = vr;
        ui[j] = vi;
      }
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        T v = tW[a * J * 2] * ur[0];
        v = fma(-tW[a * J * 2 + 1], ui[0], v);
#pragma unroll
        for (int j = 1; j < J; ++j) v = fma(tW[(a * J + j) * 2], ur[j], fma(-tW[(a * J + j) * 2 + 1], ui[j], v));
        *ep = v;
        ep += fstride;
      }
    }
  }
}

template <typename T, int D, int Q, int NT, bool DIAG>
static hipError_t vanka_tdec_impl(const LevelArgs& L, const T* Aw, const T* Bm, const T* Ft, const T* Ht,
                                  const T* tw, const T* r, T* x, T omega, T* E, hipStream_t s, bool gather,
                                  bool xzero) {
  constexpr int NL = D == 3 ? Q * Q * Q : Q * Q;
  constexpr int C = D == 3 ? (Q - 1) * Q * (Q + 1) / 6 : (Q - 1) * Q / 2;
  constexpr int MP = (NL + 15) / 16 * 16, J = (NT + 1) / 2;
  if (L.C != C || L.nloc != NL || L.nt != NT || L.N < 1 || L.N > 8 || (L.N & (L.N - 1))) return hipErrorInvalidValue;
  const int64_t ncells = L.Mp / L.C;
  const int DN = D * L.N;
  auto shm = [&](int dnp) {
    constexpr int R4 = (2 * C + 3) / 4 * 4;
    return sizeof(T) * ((size_t)J * MP * (2 * dnp + 1) + 2 * (size_t)J * 8 * R4 + (size_t)C * D * NL +
                        (size_t)NT * C * 8 + (size_t)4 * J * 16 * 17);
  };
  auto run = [&](auto kern, size_t bytes) -> hipError_t {
    if (bytes > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e != hipSuccess) return e;
    }
    kern<<<(unsigned)ncells, 256, bytes, s>>>(L, Aw, Bm, Ft, Ht, tw, r, x, omega, E, xzero ? 1 : 0);
    return hipGetLastError();
  };
  hipError_t e;
  if (DN <= 16) e = run(k_vanka_tdec<T, D, Q, NT, 1, DIAG>, shm(16));
  else if (DN <= 32) e = run(k_vanka_tdec<T, D, Q, NT, 2, DIAG>, shm(32));
  else return hipErrorInvalidValue;
  if (e != hipSuccess || !gather) return e;
  return vanka_gather<T>(L, E, x, omega, s, xzero);
}

template <typename T>
hipError_t launch_vanka_decoupled(const LevelArgs& L, const T* Aw, const T* Bm, const T* Ft, const T* Ht,
                                  const T* tw, const T* r, T* x, T omega, T* E, hipStream_t s, bool gather,
                                  bool xzero, bool diagonal) {
#define STMG_VT(DD, QQ, KK)                                                                                   \
  if (L.d == DD && L.Q == QQ && L.nt == KK)                                                                   \
    return diagonal ? vanka_tdec_impl<T, DD, QQ, KK, true>(L, Aw, Bm, Ft, Ht, tw, r, x, omega, E, s, gather, xzero) \
                    : vanka_tdec_impl<T, DD, QQ, KK, false>(L, Aw, Bm, Ft, Ht, tw, r, x, omega, E, s, gather, xzero);
  STMG_VT(2, 3, 1) STMG_VT(2, 3, 2) STMG_VT(2, 3, 3) STMG_VT(2, 3, 4)
  STMG_VT(2, 4, 1) STMG_VT(2, 4, 2) STMG_VT(2, 4, 3) STMG_VT(2, 4, 4)
  STMG_VT(3, 3, 1) STMG_VT(3, 3, 2) STMG_VT(3, 3, 3) STMG_VT(3, 3, 4)
  STMG_VT(3, 4, 1) STMG_VT(3, 4, 2) STMG_VT(3, 4, 3) STMG_VT(3, 4, 4)
#undef STMG_VT
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
__device__ __forceinline__ int64_t arr_base(const ArrLayout& A, int64_t b64) {
  if (!A.level) return b64 * A.compact_stride;
  const unsigned b = (unsigned)b64;  // array counts stay below 2^32
  const unsigned comp = b % (unsigned)A.D, t = b / (unsigned)A.D;
  const unsigned a = t % (unsigned)A.nt, n = t / (unsigned)A.nt;
  return (int64_t)n * A.slab + (int64_t)a * A.Mv + (int64_t)comp * A.nodes;
}

// out[b][..o..] (+)= sum_t M[o][t] in[b][..t..] along `axis` (nonzero range
// [lo_[o], hi_[o]) of at most MAXT taps; M stored banded and transposed,
// M[u * nout + o] = M(o, lo_[o] + u)); dims_out (dx, dy, dz), nin = extent
// of the input along the axis.  Launch: 64 x 4 threads per block, each thread
// ZC consecutive outputs along the slowest direction (z in 3D, y in 2D); grid
// (ceil(dx/64), ceil(dy/4) ceil(dz/ZC) (3D) or ceil(dy/(4 ZC)) (2D), nb).
// Taps are read unconditionally from clamped, in-bounds positions and weighted
// by zero when outside the row, so all loads of a thread are in flight together.
template <typename T, int MAXT>
__global__ __launch_bounds__(256) void k_vpass(const T* __restrict__ in, ArrLayout li, T* __restrict__ out,
                                               ArrLayout lo, int d, int axis, int dx, int dy, int dz, int nin,
                                               const T* __restrict__ M, const int* __restrict__ lo_,
                                               const int* __restrict__ hi_, int mask_in, int mask_out,
                                               int accumulate) {
  constexpr int ZC = 8;
  const int64_t b = blockIdx.z;
  const int ox = blockIdx.x * 64 + (int)(threadIdx.x & 63);
  int oy, oz0;
  if (d == 3) {
    const int ny4 = (dy + 3) / 4;
    oy = ((int)blockIdx.y % ny4) * 4 + (int)(threadIdx.x >> 6);
    oz0 = ((int)blockIdx.y / ny4) * ZC;
  } else {
    oy = ((int)blockIdx.y * 4 + (int)(threadIdx.x >> 6)) * ZC;
    oz0 = 0;
  }
  if (ox >= dx || oy >= dy) return;
  const int dims_out[3] = {dx, dy, dz};
  int dims_in[3] = {dx, dy, dz};
  dims_in[axis] = nin;
  const T* src = in + arr_base(li, b);
  T* dst = out + arr_base(lo, b);
  const int64_t strides[3] = {1, dims_in[0], (int64_t)dims_in[0] * dims_in[1]};
  const int slow = d == 3 ? 2 : 1;  // the direction walked by the thread
  T res[ZC];
  int64_t eo[ZC];
#pragma unroll
  for (int k = 0; k < ZC; ++k) {
    int o[3] = {ox, oy, oz0};
    o[slow] += k;
    res[k] = T(0);
    eo[k] = -1;
    if (o[slow] >= dims_out[slow]) continue;
    eo[k] = o[0] + (int64_t)dx * (o[1] + (int64_t)dy * o[2]);
    int64_t base = 0;
    bool in_bnd_other = false;
    for (int j = 0; j < d; ++j)
      if (j != axis) {
        base += o[j] * strides[j];
        if (mask_in && (o[j] == 0 || o[j] == dims_in[j] - 1)) in_bnd_other = true;
      }
    // along y and z the tap row is the same for the whole wave: make it uniform
    // (scalar loads of the range and the coefficients)
    const int oa = axis == 0 ? o[0] : __builtin_amdgcn_readfirstlane(o[axis]);
    const int t0 = lo_[oa], t1 = hi_[oa];
    T s = 0;
    if (!in_bnd_other && t1 > t0) {
      T mv[MAXT], xv[MAXT];
#pragma unroll
      for (int u = 0; u < MAXT; ++u) {
        const int t = min(t0 + u, t1 - 1);
        const bool on = t0 + u < t1 && !(mask_in && (t == 0 || t == nin - 1));
        mv[u] = M[u * dims_out[axis] + oa];  // banded, transposed table
        xv[u] = src[base + t * strides[axis]];
        if (!on) mv[u] = T(0);
      }
#pragma unroll
      for (int u = 0; u < MAXT; ++u) s += mv[u] * xv[u];
    }
    if (mask_out)
      for (int j = 0; j < d; ++j)
        if (o[j] == 0 || o[j] == dims_out[j] - 1) s = 0;
    res[k] = s;
  }
#pragma unroll
  for (int k = 0; k < ZC; ++k) {
    if (eo[k] < 0) continue;
    if (accumulate) dst[eo[k]] += res[k];
    else dst[eo[k]] = res[k];
  }
}

// Fused 3D velocity transfer: out_b (+)= (M x M x M) in_b for every field b,
// with M (nout x nin) banded as in k_vpass.  One work group per output brick
// BX x BY x BZ of one field: the input brick it needs (the union of the
// rows' tap ranges along every axis, e0 x e1 x e2 nodes, listed per brick
// by vtransfer_plan) is staged in LDS once, the x, y and z contractions run
// in LDS, and the output is written (or accumulated, S::ACC) once.  LDS is dynamic,
// sized by the host for the largest brick extents (VtBrick::lds_elems); a
// block lays its arrays out with its own extents.  Every contraction reads
// MAXT taps from its row's first tap on, unclamped: taps past the row carry
// zero coefficients and land on finite values (the next row, or a zeroed
// tail of MAXT - 1 rows behind each array).  The input boundary is zeroed on
// load (mask_in), the output boundary on store (mask_out).
template <int BX_, int BY_, int BZ_, bool ACC_>
struct VtBrick {
  static constexpr int BX = BX_, BY = BY_, BZ = BZ_;
  static constexpr bool ACC = ACC_;  // accumulate into the output (prolongation) or overwrite it
  // [s1: staged input + tail | y-pass output + tail] [s2: x-pass output + tail]
  static size_t s1_elems(const int* e, int maxt) {
    const size_t in = (size_t)e[0] * e[1] * e[2] + maxt, ypass = (size_t)(e[2] + maxt) * BY * BX;
    return in > ypass ? in : ypass;
  }
  static size_t lds_elems(const int* cap, int maxt) {
    return s1_elems(cap, maxt) + (size_t)(cap[2] * cap[1] + maxt) * BX;
  }
};
using VtProlong = VtBrick<32, 8, 8, true>;     // fine output, coarse input
using VtRestrict = VtBrick<16, 8, 4, false>;   // coarse output, fine input
using VtRestrictS = VtBrick<8, 8, 4, false>;   // the same with narrower bricks (h-coarsening: wider tap ranges)

// Launch geometry of k_vtransfer with the divisors it decodes block indices
// by, each with its multiplier ceil(2^32 / d) (udiv_m).  Fields b = (n, a,
// comp) of both sides are level-vector blocks (3 components, nt temporal dofs).
struct VtGrid {
  unsigned nbrick, m_nbrick, nbx, m_nbx, nbxy, m_nbxy, nt, m_nt;
  int64_t slab_in, mv_in, nodes_in, slab_out, mv_out, nodes_out;
};
// floor(v / d) for v < 2^32 / d, m = ceil(2^32 / d) (d >= 2), d = 1 passed as m = 0
__device__ __forceinline__ unsigned udiv_m(unsigned v, unsigned m) { return m ? __umulhi(v, m) : v; }

template <typename T, int MAXT, typename S>
__global__ __launch_bounds__(256) void k_vtransfer(const T* __restrict__ in, T* __restrict__ out, VtGrid G,
                                                   int nin, int nout, const T* __restrict__ M,
                                                   const int* __restrict__ tlo, int mask_in, int mask_out,
                                                   const int* __restrict__ brk) {
  constexpr int BX = S::BX, BY = S::BY, BZ = S::BZ, NOUT = BZ * BY * BX, OT = (NOUT + 255) / 256;
  constexpr int RX = 256 / BX, RZ = 256 / (BX * BY);  // rows per sweep of the x pass, z planes per sweep
  static_assert(256 % BX == 0 && 256 % (BX * BY) == 0, "brick shape");
  extern __shared__ __align__(16) unsigned char vt_raw[];
  const int tid = threadIdx.x;
  const unsigned lb = (unsigned)xcd_remap(blockIdx.x + (int64_t)gridDim.x * blockIdx.y,
                                          (int64_t)gridDim.x * gridDim.y);
  const unsigned field = udiv_m(lb, G.m_nbrick), brick = lb - field * G.nbrick;
  const unsigned kz = udiv_m(brick, G.m_nbxy), rxy = brick - kz * G.nbxy, ky = udiv_m(rxy, G.m_nbx);
  const int nbx = (int)G.nbx, nby = (int)(G.nbxy / G.nbx);
  const int kb[3] = {(int)(rxy - ky * G.nbx), (int)ky, (int)kz};
  const int o0[3] = {kb[0] * BX, kb[1] * BY, kb[2] * BZ};
  const unsigned ft = field / 3u, comp = field - 3u * ft, fn = udiv_m(ft, G.m_nt), fa = ft - fn * G.nt;
  const int on[3] = {min(BX, nout - o0[0]), min(BY, nout - o0[1]), min(BZ, nout - o0[2])};
  // staged input range of this brick along every axis
  const int i0[3] = {brk[2 * kb[0]], brk[2 * (nbx + kb[1])], brk[2 * (nbx + nby + kb[2])]};
  const int ext[3] = {brk[2 * kb[0] + 1], brk[2 * (nbx + kb[1]) + 1], brk[2 * (nbx + nby + kb[2]) + 1]};
  T* dst = out + (int64_t)fn * G.slab_out + (int64_t)fa * G.mv_out + (int64_t)comp * G.nodes_out;
  // this thread's x and y output positions (fixed for the whole block), their
  // coefficients and first taps relative to the staged range
  const int ox = tid % BX, oy = (tid / BX) % BY;
  const int gxo = o0[0] + min(ox, on[0] - 1), gyo = o0[1] + min(oy, on[1] - 1);
  T cx[MAXT], cy[MAXT];
#pragma unroll
  for (int u = 0; u < MAXT; ++u) {
    cx[u] = M[u * nout + gxo];
    cy[u] = M[u * nout + gyo];
  }
  const int offx = max(tlo[gxo] - i0[0], 0), offy = max(tlo[gyo] - i0[1], 0);
  // outputs of this thread, and (accumulating) their old values, fetched now
  int64_t gout[OT];
  T prev[OT];
#pragma unroll
  for (int e = 0; e < OT; ++e) {
    const int oz = min(tid / (BX * BY) + RZ * e, on[2] - 1);
    gout[e] = ((int64_t)(o0[2] + oz) * nout + gyo) * nout + gxo;
    prev[e] = S::ACC ? dst[gout[e]] : T(0);
  }
  T* s1 = reinterpret_cast<T*>(vt_raw);
  const int n1 = max(ext[0] * ext[1] * ext[2] + MAXT, (ext[2] + MAXT) * BY * BX);
  T* s2 = s1 + n1;
  const T* src = in + (int64_t)fn * G.slab_in + (int64_t)fa * G.mv_in + (int64_t)comp * G.nodes_in;
  // ---- stage the input brick: RW lanes per row (RW = 32 or 64), 256 / RW
  // rows of one z-plane per sweep; the sweeps (z, j) are walked uniformly,
  // CH at a time.  Offsets inside the field are 32-bit; rows past the
  // brick are read from its last row (in bounds) and not stored.
  {
    const int lrw = ext[0] <= 32 ? 5 : 6, rs = 256 >> lrw;
    const int ix = tid & ((1 << lrw) - 1), iyl = tid >> lrw;
    const int gx = i0[0] + min(ix, ext[0] - 1);
    const bool xin = ix < ext[0];
    const bool xb = (mask_in != 0) & ((gx == 0) | (gx == nin - 1));
    const int nsw = (ext[1] + rs - 1) / rs, nq = ext[2] * nsw, plane = nin * nin;
    constexpr int CH = 8;
    int iz = 0, jj = 0;  // sweep q0 = (iz, jj)
    for (int q0 = 0; q0 < nq; q0 += CH) {
      T v[CH];
      bool keep[CH];
      int z = iz, j = jj;
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        const int gy = i0[1] + min(j * rs + iyl, ext[1] - 1), gz = i0[2] + min(z, ext[2] - 1);
        const bool zb = (gz == 0) | (gz == nin - 1), yb = (gy == 0) | (gy == nin - 1);
        keep[e] = !(xb | ((mask_in != 0) & (yb | zb)));
        v[e] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(src) +
                                           (unsigned)(gz * plane + gy * nin + gx) * (unsigned)sizeof(T));
        if (++j == nsw) {
          j = 0;
          ++z;
        }
      }
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        const int iy = jj * rs + iyl;
        if ((q0 + e < nq) & xin & (iy < ext[1])) s1[(iz * ext[1] + iy) * ext[0] + ix] = keep[e] ? v[e] : T(0);
        if (++jj == nsw) {
          jj = 0;
          ++iz;
        }
      }
    }
    if (tid < MAXT) s1[ext[0] * ext[1] * ext[2] + tid] = T(0);
  }
  __syncthreads();
  // ---- x: s2[row][ox], row = (iz, iy)
  {
    const int nrow = ext[1] * ext[2];
    if (ox < on[0])
      for (int row = tid / BX; row < nrow; row += RX) {
        const T* p = s1 + row * ext[0] + offx;
        T sum = 0;
#pragma unroll
        for (int u = 0; u < MAXT; ++u) sum += cx[u] * p[u];
        s2[row * BX + ox] = sum;
      }
    if (tid < MAXT * BX) s2[nrow * BX + tid] = T(0);
  }
  __syncthreads();
  // ---- y: s1[iz][oy][ox]
  {
    if (ox < on[0] && oy < on[1])
      for (int iz = tid / (BX * BY); iz < ext[2]; iz += RZ) {
        const T* p = s2 + (iz * ext[1] + offy) * BX + ox;
        T sum = 0;
#pragma unroll
        for (int u = 0; u < MAXT; ++u) sum += cy[u] * p[u * BX];
        s1[(iz * BY + oy) * BX + ox] = sum;
      }
    for (int t = tid; t < MAXT * BY * BX; t += 256) s1[ext[2] * BY * BX + t] = T(0);
  }
  __syncthreads();
  // ---- z, then the output brick (the z position is uniform over a wave)
#pragma unroll
  for (int e = 0; e < OT; ++e) {
    const int oz = __builtin_amdgcn_readfirstlane(tid / (BX * BY) + RZ * e);
    if (oz < on[2] && ox < on[0] && oy < on[1]) {
      const int gz = o0[2] + oz, offz = max(tlo[gz] - i0[2], 0);
      const T* p = s1 + (offz * BY + oy) * BX + ox;
      T sum = 0;
#pragma unroll
      for (int u = 0; u < MAXT; ++u) sum += M[u * nout + gz] * p[u * BY * BX];
      if (mask_out && (gxo == 0 || gxo == nout - 1 || gyo == 0 || gyo == nout - 1 || gz == 0 || gz == nout - 1))
        sum = 0;
      dst[gout[e]] = S::ACC ? prev[e] + sum : sum;
    }
  }
}

// Pressure: prolong (dir 0): xf[cf][l] += sum_m E[pos][l][m] xc[parent][m];
// restrict (dir 1): bc[cp][m] = sum_children sum_l E[pos][l][m] rf[child][l].
template <typename T>
__global__ void k_ppass(const T* __restrict__ in, T* __restrict__ out, int nslices, int nt_in, int nt_out,
                        int64_t slab_in, int64_t off_in, int64_t Mp_in, int64_t slab_out, int64_t off_out,
                        int64_t Mp_out, int d, int n_out, int n_in, int C_out, int C_in, const T* __restrict__ E,
                        int npos, int dir, int Cf, int Cc) {
  // 32-bit index arithmetic: the launchers keep nslices * ncell * C_out below 2^31
  const unsigned no = (unsigned)n_out, ncell = d == 3 ? no * no * no : no * no;
  const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (unsigned)nslices * ncell * (unsigned)C_out) return;
  const unsigned l = idx % (unsigned)C_out, q = idx / (unsigned)C_out, c = q % ncell, s = q / ncell;
  const int n = (int)(s / (unsigned)nt_out), a = (int)(s % (unsigned)nt_out);
  const unsigned rr = c / no;
  const int cc[3] = {(int)(c - rr * no), (int)(d == 3 ? rr % no : rr), (int)(d == 3 ? rr / no : 0u)};
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


// taps per contraction of the fused transfer kernel (its MAXT) for rows of up
// to max_row taps
static int vt_taps(int max_row) { return max_row <= 3 ? 3 : (max_row <= 5 ? 5 : (max_row <= 7 ? 7 : 8)); }

// staged input range (first node, extent) of every output brick of `b` rows
// along one axis, appended to `out`; returns the largest extent
static int brick_ranges(const std::vector<int>& lo, const std::vector<int>& hi, int b, std::vector<int>& out) {
  const int nout = (int)lo.size();
  int worst = 1;
  for (int o0 = 0; o0 < nout; o0 += b) {
    int a = 0x7fffffff, e = -1;
    for (int o = o0; o < std::min(o0 + b, nout); ++o)
      if (hi[o] > lo[o]) {
        a = std::min(a, lo[o]);
        e = std::max(e, hi[o]);
      }
    if (e <= a) {  // no tap in the brick
      a = 0;
      e = 1;
    }
    out.push_back(a);
    out.push_back(e - a);
    worst = std::max(worst, e - a);
  }
  return worst;
}

template <typename S>
static size_t vt_plan_bytes(const std::vector<int>& lo, const std::vector<int>& hi, int max_row, size_t elem,
                            int* cap, std::vector<int>& brk) {
  brk.clear();
  cap[0] = brick_ranges(lo, hi, S::BX, brk);
  cap[1] = brick_ranges(lo, hi, S::BY, brk);
  cap[2] = brick_ranges(lo, hi, S::BZ, brk);
  if (cap[0] > 64 || cap[1] > 64 || cap[2] > 64) return ~(size_t)0;
  return S::lds_elems(cap, vt_taps(max_row)) * elem;
}

int vtransfer_plan(const std::vector<int>& lo, const std::vector<int>& hi, int d, int max_row, bool restriction,
                   size_t elem, int* cap, std::vector<int>& brk) {
  if (d != 3 || max_row > 8) return 0;
  if (!restriction) return vt_plan_bytes<VtProlong>(lo, hi, max_row, elem, cap, brk) <= 48 * 1024 ? 1 : 0;
  if (vt_plan_bytes<VtRestrict>(lo, hi, max_row, elem, cap, brk) <= 40 * 1024) return 2;
  if (vt_plan_bytes<VtRestrictS>(lo, hi, max_row, elem, cap, brk) <= 56 * 1024) return 3;
  return 0;
}

namespace {
unsigned udiv_mult(unsigned d) { return d <= 1 ? 0u : (unsigned)((0x100000000ULL + d - 1) / d); }

template <typename T, typename S>
void launch_vt(const T* in, ArrLayout li, T* out, ArrLayout lo, int nin, int nout, int64_t nb, int max_row,
               const T* M, const int* tlo, int mask_in, int mask_out, const int* cap, const int* brk,
               hipStream_t s) {
  VtGrid G;
  G.nbx = (unsigned)((nout + S::BX - 1) / S::BX);
  G.nbxy = G.nbx * (unsigned)((nout + S::BY - 1) / S::BY);
  G.nbrick = G.nbxy * (unsigned)((nout + S::BZ - 1) / S::BZ);
  G.nt = (unsigned)li.nt;
  G.m_nbrick = udiv_mult(G.nbrick);
  G.m_nbx = udiv_mult(G.nbx);
  G.m_nbxy = udiv_mult(G.nbxy);
  G.m_nt = udiv_mult(G.nt);
  G.slab_in = li.slab; G.mv_in = li.Mv; G.nodes_in = li.nodes;
  G.slab_out = lo.slab; G.mv_out = lo.Mv; G.nodes_out = lo.nodes;
  const dim3 grid(G.nbrick, (unsigned)nb);
  const int taps = vt_taps(max_row);
  const size_t bytes = S::lds_elems(cap, taps) * sizeof(T);
  auto go = [&](auto kern) {
    kern<<<grid, 256, bytes, s>>>(in, out, G, nin, nout, M, tlo, mask_in, mask_out, brk);
  };
  if (taps == 3) go(k_vtransfer<T, 3, S>);
  else if (taps == 5) go(k_vtransfer<T, 5, S>);
  else if (taps == 7) go(k_vtransfer<T, 7, S>);
  else go(k_vtransfer<T, 8, S>);
}
}  // namespace

template <typename T>
static void space_velocity(const LevelArgs& Li, const LevelArgs& Lo, int nt, int N, const T* M, const int* lo,
                           const int* hi, int max_row, int brick, const int* cap, const int* brk, const T* in,
                           ArrLayout li, T* out, ArrLayout lout, T* tmp1, T* tmp2, bool restrict_, hipStream_t s) {
  // Li: spatial sizes of the input, Lo: of the output.  Prolongation runs the
  // passes x, y, z and restriction z, y, x, so that the x pass (whose taps
  // differ from lane to lane) always works on the coarse side of the
  // intermediate arrays.
  const int d = Li.d;
  const int64_t nb = (int64_t)N * nt * d;
  if (brick > 0 && d == 3 && li.level && lout.level && li.nt == lout.nt) {  // one fused launch
    const int mi = 1, mo = restrict_ ? 1 : 0;  // prolongation accumulates (VtProlong::ACC)
    if (brick == 1)
      launch_vt<T, VtProlong>(in, li, out, lout, Li.nn, Lo.nn, nb, max_row, M, lo, mi, mo, cap, brk, s);
    else if (brick == 2)
      launch_vt<T, VtRestrict>(in, li, out, lout, Li.nn, Lo.nn, nb, max_row, M, lo, mi, mo, cap, brk, s);
    else
      launch_vt<T, VtRestrictS>(in, li, out, lout, Li.nn, Lo.nn, nb, max_row, M, lo, mi, mo, cap, brk, s);
    return;
  }
  int dims[3] = {Li.nn, Li.nn, d == 3 ? Li.nn : 1};
  const T* src = in;
  ArrLayout ls = li;
  for (int pass = 0; pass < d; ++pass) {
    const int axis = restrict_ ? d - 1 - pass : pass;
    int nin = dims[axis];
    dims[axis] = Lo.nn;
    bool last = pass == d - 1;
    T* dst = last ? out : (pass == 0 ? tmp1 : tmp2);
    ArrLayout ld = lout;
    if (!last) {
      ld.level = 0;
      ld.compact_stride = (int64_t)dims[0] * dims[1] * dims[2];
    }
    const unsigned gy = d == 3 ? (unsigned)(((dims[1] + 3) / 4) * ((dims[2] + 7) / 8))
                               : (unsigned)((dims[1] + 31) / 32);
    const dim3 grid(nblk(dims[0], 64), gy, (unsigned)nb);
    const int mi = pass == 0 ? 1 : 0, mo = (last && restrict_) ? 1 : 0, acc = (last && !restrict_) ? 1 : 0;
    if (max_row <= 4)
      k_vpass<T, 4><<<grid, 256, 0, s>>>(src, ls, dst, ld, d, axis, dims[0], dims[1], dims[2], nin, M, lo, hi, mi,
                                          mo, acc);
    else if (max_row <= 8)
      k_vpass<T, 8><<<grid, 256, 0, s>>>(src, ls, dst, ld, d, axis, dims[0], dims[1], dims[2], nin, M, lo, hi, mi,
                                          mo, acc);
    else
      k_vpass<T, 16><<<grid, 256, 0, s>>>(src, ls, dst, ld, d, axis, dims[0], dims[1], dims[2], nin, M, lo, hi, mi,
                                           mo, acc);
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
  space_velocity<T>(Cs, F, F.nt, F.N, P1, rlo, rhi, t.max_row_p1, t.vt_p1, t.cap_p1, t.brk_p1, src, li, xf, lo,
                    tmp1, tmp2, false, s);
  int64_t tot = (int64_t)F.N * F.nt * (int64_t)(F.Mp);
  if (tot >= (int64_t)1 << 31) return hipErrorInvalidValue;
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
  space_velocity<T>(F, Cs, F.nt, F.N, P1T, clo, chi, t.max_row_p1t, t.vt_p1t, t.cap_p1t, t.brk_p1t, rf, li, dst,
                    lo, tmp1, tmp2, true, s);
  int64_t ncc = 1;
  for (int j = 0; j < F.d; ++j) ncc *= Cs.n;
  int64_t tot = (int64_t)F.N * F.nt * ncc * Cs.C;
  if (tot >= (int64_t)1 << 31) return hipErrorInvalidValue;
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

// <r, w>, <w, w>, <r, r> in one pass (FP64 accumulation, fixed order)
template <typename T>
__global__ __launch_bounds__(256) void k_dot3(const T* __restrict__ r, const T* __restrict__ w, int64_t n,
                                              double* __restrict__ partial) {
  __shared__ double sh[4];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double a = (double)r[i], b = (double)w[i];
    s0 += a * b;
    s1 += b * b;
    s2 += a * a;
  }
  s0 = block_sum(s0, sh);
  __syncthreads();
  s1 = block_sum(s1, sh);
  __syncthreads();
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s0;
    partial[kDotBlocks + blockIdx.x] = s1;
    partial[2 * kDotBlocks + blockIdx.x] = s2;
  }
}
template <typename T>
hipError_t launch_dot3(const T* r, const T* w, int64_t n, double* partial, double* out, hipStream_t s) {
  k_dot3<T><<<kDotBlocks, 256, 0, s>>>(r, w, n, partial);
  k_dot_final<<<1, 64, 0, s>>>(partial, 3, out);
  return hipGetLastError();
}
template hipError_t launch_dot3<double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template hipError_t launch_dot3<float>(const float*, const float*, int64_t, double*, double*, hipStream_t);

// ---- Gram-Schmidt passes of the Arnoldi process (lagged CGS2), templated on
// a bound NVM of the number of basis vectors (per-thread accumulators; the
// basis values of one element are kept in registers for NVM <= 32 and read
// again otherwise), kFusedBlocks blocks, sums in a fixed order.  Two work
// groups per compute unit: with 13-16 basis vectors read side by side, fewer
// streams in flight ran 4% faster than eight work groups per unit.
constexpr int kFusedBlocks = 512;

// Sums of nv values over a block, written to partial[k * kFusedBlocks + block].
template <int NA>
__device__ __forceinline__ void block_sums_out(const double (&acc)[NA], int nv, double* sh, double* partial) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64, nw = blockDim.x / 64;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    if (k >= nv) continue;
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[k * 4 + wv] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nv; k += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += sh[k * 4 + i];
    partial[(int64_t)k * kFusedBlocks + blockIdx.x] = s;
  }
}

// Both passes read NVM basis vectors per element unconditionally, in
// chunks of up to 16 whose loads are all in flight together: vector k >=
// (number in use) is read from the last one in use (an L1/L2 hit) and
// weighted by zero (predicated loads would each be followed by a full wait).
// NVM runs in steps of 4 up to 32, so at most 3 such reads per element.
constexpr int kCgsChunk = 16;

// First pass of a step with j final basis vectors V_0..V_{j-1} and a pending
// vector u with second-projection coefficients h2 and norm 1/invb:
//   V_j = (u - sum_{k<j} h2_k V_k) invb   (written; skipped when pending == 0)
//   partial sums of V_k . w for k <= j (k < j when pending == 0).
template <int NVM>
__global__ __launch_bounds__(256) void k_lcgs_a(double* __restrict__ V, int64_t ldv, int j, int pending,
                                                const double* __restrict__ u, const double* __restrict__ h2,
                                                double invb, const double* __restrict__ w, int64_t n,
                                                double* __restrict__ partial) {
  __shared__ double sh[NVM * 4];
  const int nf = pending ? j : j + 1;  // final vectors read (>= 1)
  double acc[NVM];
#pragma unroll
  for (int k = 0; k < NVM; ++k) acc[k] = 0.0;
  double* vj = V + (int64_t)j * ldv;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = w[i];
    const double ui = pending ? u[i] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NVM; c += kCgsChunk) {
      constexpr int CN = NVM < kCgsChunk ? NVM : kCgsChunk;
      double v[CN];
#pragma unroll
      for (int k = 0; k < CN; ++k) v[k] = V[(int64_t)min(c + k, nf - 1) * ldv + i];
#pragma unroll
      for (int k = 0; k < CN; ++k) {
        const bool in = c + k < nf;
        s += (pending && in ? h2[c + k] : 0.0) * v[k];
        acc[c + k] += (in ? 1.0 : 0.0) * (v[k] * wi);
      }
    }
    if (pending) {
      const double vn = (ui - s) * invb;
      vj[i] = vn;
#pragma unroll
      for (int k = 0; k < NVM; ++k) acc[k] += (k == j ? 1.0 : 0.0) * (vn * wi);
    }
  }
  block_sums_out<NVM>(acc, j + 1, sh, partial);
}

// Second pass: w -= sum_{k<nv} h_k V_k (also rounded to FP32 into w32 when
// given), then partial sums of V_k . w (updated w) for k < nv and of w . w
// (index nv).  The basis values stay in registers
// up to 16 vectors; beyond, the second use reads them again (L2).
template <int NVM>
__global__ __launch_bounds__(256) void k_axpy_mdot(double* __restrict__ w, const double* __restrict__ V,
                                                   int64_t ldv, int nv, const double* __restrict__ h, int64_t n,
                                                   double* __restrict__ partial, float* __restrict__ w32) {
  constexpr bool KEEP = NVM <= kCgsChunk;
  constexpr int CN = NVM < kCgsChunk ? NVM : kCgsChunk;
  __shared__ double sh[(NVM + 1) * 4];
  double acc[NVM + 1];
#pragma unroll
  for (int k = 0; k <= NVM; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double w0 = w[i];
    double v[CN];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NVM; c += kCgsChunk) {
#pragma unroll
      for (int k = 0; k < CN; ++k) v[k] = V[(int64_t)min(c + k, nv - 1) * ldv + i];
#pragma unroll
      for (int k = 0; k < CN; ++k) s += (c + k < nv ? h[c + k] : 0.0) * v[k];
    }
    const double wi = w0 - s;
    w[i] = wi;
    if (w32) w32[i] = (float)wi;  // the next direction in FP32 (the mixed V-cycle's input)
#pragma unroll
    for (int c = 0; c < NVM; c += kCgsChunk) {
      if constexpr (!KEEP) {
#pragma unroll
        for (int k = 0; k < CN; ++k) v[k] = V[(int64_t)min(c + k, nv - 1) * ldv + i];
      }
#pragma unroll
      for (int k = 0; k < CN; ++k) acc[c + k] += (c + k < nv ? 1.0 : 0.0) * (v[k] * wi);
    }
    acc[NVM] += wi * wi;
  }
  // move the norm next to the nv dot products
  double out[NVM + 1];
#pragma unroll
  for (int k = 0; k <= NVM; ++k) out[k] = k == nv ? acc[NVM] : acc[k];
  block_sums_out<NVM + 1>(out, nv + 1, sh, partial);
}

// out[v] = sum of the kFusedBlocks partial sums of vector v: one 256-thread
// block per vector, each thread a strided eighth of them, then a fixed tree
// over the block (the order never changes, so results are reproducible).
__global__ __launch_bounds__(256) void k_fused_final(const double* __restrict__ partial, int nv,
                                                     double* __restrict__ out) {
  static_assert(kFusedBlocks % 256 == 0, "partial layout");
  __shared__ double sh[4];
  const int vi = blockIdx.x;
  if (vi >= nv) return;
  const double* p = partial + (int64_t)vi * kFusedBlocks + threadIdx.x;
  double v[kFusedBlocks / 256];
#pragma unroll
  for (int k = 0; k < kFusedBlocks / 256; ++k) v[k] = p[256 * k];
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kFusedBlocks / 256; ++k) s += v[k];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[vi] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

template <int NVM>
static void lcgs2_impl(double* V, int64_t ldv, int j, int pending, const double* u, const double* h2_prev,
                       double invb, double* w, int64_t n, double* partial, double* h1, double* h2n,
                       float* w32, hipStream_t s) {
  const int nv = j + 1;
  k_lcgs_a<NVM><<<kFusedBlocks, 256, 0, s>>>(V, ldv, j, pending, u, h2_prev, invb, w, n, partial);
  k_fused_final<<<nv, 256, 0, s>>>(partial, nv, h1);
  k_axpy_mdot<NVM><<<kFusedBlocks, 256, 0, s>>>(w, V, ldv, nv, h1, n, partial, w32);
  k_fused_final<<<nv + 1, 256, 0, s>>>(partial, nv + 1, h2n);
}

hipError_t launch_lcgs2(double* V, int64_t ldv, int j, int pending, const double* u, const double* h2_prev,
                        double invb, double* w, int64_t n, double* partial, double* h1, double* h2n, float* w32,
                        hipStream_t s) {
  const int nv = j + 1;
  if (j < 0 || nv > kMaxFused || (!pending && j != 0)) return hipErrorInvalidValue;
#define STMG_LC(K) \
  if (nv <= K) {   \
    lcgs2_impl<K>(V, ldv, j, pending, u, h2_prev, invb, w, n, partial, h1, h2n, w32, s); \
    return hipGetLastError();                                                     \
  }
  STMG_LC(4) STMG_LC(8) STMG_LC(12) STMG_LC(16) STMG_LC(20) STMG_LC(24) STMG_LC(28) STMG_LC(32)
  STMG_LC(40) STMG_LC(48) STMG_LC(56) STMG_LC(64)
#undef STMG_LC
  return hipGetLastError();
}

// w += sign sum_k h_k V_k (assign: w = sign sum_k h_k V_k, w not read)
__global__ void k_multi_axpy(double* __restrict__ w, const double* __restrict__ V, int64_t ldv, int nv,
                             const double* __restrict__ h, int64_t n, double sign, int assign) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nv; ++k) s += h[k] * V[(int64_t)k * ldv + i];
  w[i] = (assign ? 0.0 : w[i]) + sign * s;
}
hipError_t launch_multi_axpy(double* w, const double* V, int64_t ldv, int nv, const double* h, int64_t n,
                             hipStream_t s) {
  k_multi_axpy<<<nblk(n), 256, 0, s>>>(w, V, ldv, nv, h, n, -1.0, 0);
  return hipGetLastError();
}
hipError_t launch_combine(double* x, const double* Z, int64_t ldz, int nv, const double* y, int64_t n,
                          hipStream_t s, bool assign) {
  k_multi_axpy<<<nblk(n), 256, 0, s>>>(x, Z, ldz, nv, y, n, 1.0, assign ? 1 : 0);
  return hipGetLastError();
}
__global__ void k_combine_f32(double* __restrict__ x, const float* __restrict__ Z, int64_t ldz, int nv,
                              const double* __restrict__ y, int64_t n, int assign) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // 8 basis loads in flight at a time (indices past nv read the last vector, weight 0)
  double s = 0.0;
  for (int k0 = 0; k0 < nv; k0 += 8) {
    float z[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) z[k] = Z[(int64_t)min(k0 + k, nv - 1) * ldz + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += (k0 + k < nv ? y[k0 + k] : 0.0) * (double)z[k];
  }
  x[i] = (assign ? 0.0 : x[i]) + s;
}
hipError_t launch_combine_f32(double* x, const float* Z, int64_t ldz, int nv, const double* y, int64_t n,
                              hipStream_t s, bool assign) {
  k_combine_f32<<<nblk(n), 256, 0, s>>>(x, Z, ldz, nv, y, n, assign ? 1 : 0);
  return hipGetLastError();
}
__global__ void k_scale_copy(double* y, const double* x, double inv, int64_t n, float* y32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i] * inv;
  y[i] = v;
  if (y32) y32[i] = (float)v;
}
hipError_t launch_scale_copy(double* y, const double* x, double inv, int64_t n, hipStream_t s, float* y32) {
  k_scale_copy<<<nblk(n), 256, 0, s>>>(y, x, inv, n, y32);
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
  template hipError_t launch_apply<T>(const LevelArgs&, const T*, const T*, const T*, const T*, T*, int, T*,      \
                                      hipStream_t, bool, int, int);                                                 \
  template hipError_t launch_vanka_factored<T>(const LevelArgs&, const T*, const T*, const T*, const T*, const T*, \
                                               const T*, T*, T, T*, hipStream_t, bool, bool);                       \
  template hipError_t launch_vanka_dense<T>(const LevelArgs&, const T*, const T*, T*, T, hipStream_t);             \
  template hipError_t launch_vanka_decoupled<T>(const LevelArgs&, const T*, const T*, const T*, const T*,          \
                                                const T*, const T*, T*, T, T*, hipStream_t, bool, bool, bool);      \
  template hipError_t launch_prolongate_add<T>(const LevelArgs&, const LevelArgs&, const TransferDev&, const T*,   \
                                               const int*, const int*, const T*, const T*, const T*, T*, T*, T*,    \
                                               T*, hipStream_t);                                                    \
  template hipError_t launch_restrict<T>(const LevelArgs&, const LevelArgs&, const TransferDev&, const T*,         \
                                         const int*, const int*, const T*, const T*, const T*, T*, T*, T*, T*,      \
                                         hipStream_t);                                                              \
  template hipError_t launch_vanka_gather_only<T>(const LevelArgs&, const T*, T*, T, hipStream_t, bool);                \
  template hipError_t launch_coarse<T>(int64_t, int64_t, int, int, const double*, const double*, const T*, T*,  \
                                        hipStream_t);                          \
  template hipError_t launch_fill<T>(T*, T, int64_t, hipStream_t);                                                  \
  template hipError_t launch_axpy<T>(T*, T, const T*, int64_t, hipStream_t);
STMG_INST(double)
STMG_INST(float)
#undef STMG_INST

}  // namespace stmg
