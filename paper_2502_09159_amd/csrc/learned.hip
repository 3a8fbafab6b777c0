// Learned correction network on gfx950: BF16 16x16x16 MFMA with FP32
// accumulation.  Activations are stored per sample as 32 rows (27 nodes of
// the 3x3x3 grid, padded) x C channels (padded to 16 or 32).  A convolution
// layer is out[p] = sum_o in[nbr(o, p)] W_o (27 shifted GEMMs); its data
// gradient is the same operation with the flipped, transposed weights.
#include <hip/hip_runtime.h>

#include "learned.hpp"

namespace stmg {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int G = 8;  // samples per work group (256 threads, 4 waves)

__device__ __forceinline__ uint16_t to_bf16(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);  // round to nearest even (one instruction on gfx950)
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// neighbour of position p (x fastest on 3x3x3) at offset o, or -1
__device__ __forceinline__ int nbr(int o, int p) {
  if (p >= 27) return -1;
  int x = p % 3 + o % 3 - 1, y = (p / 3) % 3 + (o / 3) % 3 - 1, z = p / 9 + o / 9 - 1;
  if (x < 0 || x > 2 || y < 0 || y > 2 || z < 0 || z > 2) return -1;
  return x + 3 * y + 9 * z;
}

// sizes of the fragment blocks: forward layers 1..3, then transposed 3 and 2
__host__ __device__ constexpr int frag_elems(int cip, int cop) { return 27 * (cip / 16) * (cop / 16) * 256; }
constexpr int F1 = frag_elems(16, 32), F2 = frag_elems(32, 32), F3 = frag_elems(32, 16);
constexpr int OFF_W1 = 0, OFF_W2 = 32 * 15 * 27, OFF_W3 = OFF_W2 + 32 * 32 * 27;

// One convolution over the G samples in LDS: out[g][p][co] = sum_o sum_ci in[g][nbr(o,p)][ci] W.
// frag: B operands, ((o KB + kb) CT + ct) 64 + lane, 4 BF16 each.
// MODE 0: ReLU -> BF16 out (LDS);  1: FP32 out (LDS);  2: x relu'(act) -> BF16 out
// RSI / RSO: row strides (elements) of in and out (act has out's layout)
template <int CIP, int COP, int MODE, int GS = G, int RSI = CIP, int RSO = COP>
__device__ void conv_block(const uint16_t* __restrict__ in, const bf16x4* __restrict__ frag, void* out,
                           const uint16_t* __restrict__ act) {
  constexpr int KB = CIP / 16, CT = COP / 16, RT = GS * 2;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  f32x4 acc[RT / 4][CT];
#pragma unroll
  for (int it = 0; it < RT / 4; ++it)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[it][ct] = f32x4{0, 0, 0, 0};
  // a wave's row tiles rt = wave + 4 it all have rt % 2 == wave % 2, so the
  // lane's position p, and its neighbour at offset o, do not depend on it
  const int p = (wave % 2) * 16 + lane % 16;
  // The offsets are unrolled, so that the loads of later offsets are issued
  // ahead of the matrix products of earlier ones.  A missing neighbour reads
  // row 27 of the sample, a padding row: every activation and gradient array
  // keeps rows 27..31 at zero (the network inputs and the loss gradient are
  // written so, and conv_block writes zeros there).  Bit o of nb is set when
  // position p has a neighbour at offset o.
  int nb = 0;
#pragma unroll
  for (int o = 0; o < 27; ++o) nb |= (nbr(o, p) >= 0 ? 1 : 0) << o;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int shift = (o % 3 - 1) + 3 * ((o / 3) % 3 - 1) + 9 * (o / 9 - 1);
    const int q = (nb >> o) & 1 ? p + shift : 27;
    const uint16_t* row = in + q * RSI + 4 * (lane / 16);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      bf16x4 b[CT], a[RT / 4];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) b[ct] = frag[((o * KB + kb) * CT + ct) * 64 + lane];
#pragma unroll
      for (int it = 0; it < RT / 4; ++it)
        a[it] = *reinterpret_cast<const bf16x4*>(row + ((wave + 4 * it) / 2) * 32 * RSI + kb * 16);
#pragma unroll
      for (int it = 0; it < RT / 4; ++it)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          acc[it][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[it], b[ct], acc[it][ct], 0, 0, 0);
    }
  }
#pragma unroll
  for (int it = 0; it < RT / 4; ++it) {
    const int rt = wave + 4 * it;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rt * 16 + 4 * (lane / 16) + v;  // g * 32 + p
        const int p = row % 32, co = ct * 16 + lane % 16;
        float val = p < 27 ? acc[it][ct][v] : 0.0f;
        if (MODE == 0) {
          static_cast<uint16_t*>(out)[row * RSO + co] = to_bf16(fmaxf(val, 0.0f));
        } else if (MODE == 1) {
          static_cast<float*>(out)[row * RSO + co] = val;
        } else {
          float d = from_bf16(act[row * RSO + co]) > 0.0f ? val : 0.0f;
          static_cast<uint16_t*>(out)[row * RSO + co] = to_bf16(d);
        }
      }
  }
}

// ------------------------------------------------------------ forward
// x: [s][32][16] BF16 -> h1, h2 [s][32][32] BF16 (optional) -> y [s][32][16] FP32
// Inference only (no activations kept): GI samples per work group, with two
// LDS regions reused layer by layer (A: h1, then y; B: x, then h2), so that
// twice the samples share each weight fragment a wave reads.  BF16 rows are
// padded by 4 elements (8 bytes): the 16 positions a wave reads at once then
// start in 16 different LDS banks (unpadded 32- and 64-byte rows put 4 or 8
// of them on the same bank).
constexpr int GI = 16, RS16 = 16 + 4, RS32 = 32 + 4;
__global__ __launch_bounds__(256, 2) void k_net_infer(const uint16_t* __restrict__ x, const bf16x4* __restrict__ fw,
                                                   float* __restrict__ y, int64_t count) {
  static_assert(GI * 32 * 16 * sizeof(float) <= GI * 32 * RS32 * sizeof(uint16_t), "region A holds h1, then y");
  __shared__ __align__(16) uint16_t sA[GI * 32 * RS32];
  __shared__ __align__(16) uint16_t sB[GI * 32 * RS32];
  const int64_t s0 = (int64_t)blockIdx.x * GI;
  const int ns = (int)min<int64_t>(GI, count - s0);
  // x rows of 16 BF16 as 4 chunks of 8 bytes
  for (int t = threadIdx.x; t < GI * 32 * 4; t += blockDim.x) {
    const int row = t / 4, c4 = t % 4;
    const unsigned long long v =
        (row / 32) < ns ? reinterpret_cast<const unsigned long long*>(x + s0 * 512)[t] : 0ull;
    *reinterpret_cast<unsigned long long*>(sB + row * RS16 + 4 * c4) = v;
  }
  __syncthreads();
  conv_block<16, 32, 0, GI, RS16, RS32>(sB, fw, sA, nullptr);
  __syncthreads();
  conv_block<32, 32, 0, GI, RS32, RS32>(sA, fw + F1 / 4, sB, nullptr);
  __syncthreads();
  float* sy = reinterpret_cast<float*>(sA);
  conv_block<32, 16, 1, GI, RS32, 16>(sB, fw + (F1 + F2) / 4, sy, nullptr);
  __syncthreads();
  for (int t = threadIdx.x; t < ns * 512; t += blockDim.x) y[s0 * 512 + t] = sy[t];
}

// Training forward: keeps the hidden activations for the backward pass.
__global__ __launch_bounds__(256) void k_net_fwd(const uint16_t* __restrict__ x, const bf16x4* __restrict__ fw,
                                                 uint16_t* __restrict__ h1g, uint16_t* __restrict__ h2g,
                                                 float* __restrict__ y, int64_t count) {
  __shared__ __align__(16) uint16_t sx[G * 32 * 16];
  __shared__ __align__(16) uint16_t sh1[G * 32 * 32];
  __shared__ __align__(16) uint16_t sh2[G * 32 * 32];
  __shared__ __align__(16) float sy[G * 32 * 16];
  const int64_t s0 = (int64_t)blockIdx.x * G;
  const int ns = (int)min<int64_t>(G, count - s0);
  for (int t = threadIdx.x; t < G * 32 * 16; t += blockDim.x) sx[t] = (t / 512) < ns ? x[s0 * 512 + t] : 0;
  __syncthreads();
  conv_block<16, 32, 0>(sx, fw, sh1, nullptr);
  __syncthreads();
  conv_block<32, 32, 0>(sh1, fw + F1 / 4, sh2, nullptr);
  __syncthreads();
  conv_block<32, 16, 1>(sh2, fw + (F1 + F2) / 4, sy, nullptr);
  __syncthreads();
  for (int t = threadIdx.x; t < ns * 512; t += blockDim.x) y[s0 * 512 + t] = sy[t];
  if (h1g)
    for (int t = threadIdx.x; t < ns * 1024; t += blockDim.x) {
      h1g[s0 * 1024 + t] = sh1[t];
      h2g[s0 * 1024 + t] = sh2[t];
    }
}

// ------------------------------------------------------------ backward
// dy [s][32][16] BF16 (unscaled 2 (head - t) chain), activations saved by the
// forward pass; writes the per-work-group weight gradient (ABI order) to partial.
template <int CIP, int COP>
__device__ void weight_grad(const uint16_t* __restrict__ in, const uint16_t* __restrict__ dout, float* __restrict__ pw,
                            int cin, int cout) {
  // dW[co][ci][o] = sum_{g,p} in[g][nbr(o,p)][ci] dout[g][p][co]  as D(ci x co) = A(ci x k) B(k x co)
  constexpr int KB = CIP / 16, CT = COP / 16, KS = G * 32 / 16;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int tile = wave; tile < 27 * KB * CT; tile += 4) {
    const int o = tile / (KB * CT), cb = (tile / CT) % KB, ct = tile % CT;
    f32x4 acc = f32x4{0, 0, 0, 0};
    for (int ks = 0; ks < KS; ++ks) {
      bf16x4 a, b;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = ks * 16 + 4 * (lane / 16) + j;  // row g*32 + p
        const int g = k / 32, p = k % 32, q = nbr(o, p);
        a[j] = q >= 0 ? (short)in[(g * 32 + q) * CIP + cb * 16 + lane % 16] : (short)0;
        b[j] = (short)dout[k * COP + ct * 16 + lane % 16];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ci = cb * 16 + 4 * (lane / 16) + v, co = ct * 16 + lane % 16;
      if (ci < cin && co < cout) pw[((int64_t)co * cin + ci) * 27 + o] = acc[v];
    }
  }
}

__global__ __launch_bounds__(256) void k_net_bwd(const uint16_t* __restrict__ x, const uint16_t* __restrict__ h1g,
                                                 const uint16_t* __restrict__ h2g, const uint16_t* __restrict__ dyg,
                                                 const bf16x4* __restrict__ bw, float* __restrict__ partial,
                                                 int64_t count) {
  __shared__ __align__(16) uint16_t sx[G * 32 * 16];
  __shared__ __align__(16) uint16_t sh1[G * 32 * 32];
  __shared__ __align__(16) uint16_t sh2[G * 32 * 32];
  __shared__ __align__(16) uint16_t sdy[G * 32 * 16];
  __shared__ __align__(16) uint16_t sd2[G * 32 * 32];
  __shared__ __align__(16) uint16_t sd1[G * 32 * 32];
  const int64_t s0 = (int64_t)blockIdx.x * G;
  const int ns = (int)min<int64_t>(G, count - s0);
  for (int t = threadIdx.x; t < G * 512; t += blockDim.x) {
    bool ok = (t / 512) < ns;
    sx[t] = ok ? x[s0 * 512 + t] : 0;
    sdy[t] = ok ? dyg[s0 * 512 + t] : 0;
  }
  for (int t = threadIdx.x; t < G * 1024; t += blockDim.x) {
    bool ok = (t / 1024) < ns;
    sh1[t] = ok ? h1g[s0 * 1024 + t] : 0;
    sh2[t] = ok ? h2g[s0 * 1024 + t] : 0;
  }
  __syncthreads();
  float* pw = partial + (int64_t)blockIdx.x * kNetParams;
  weight_grad<32, 16>(sh2, sdy, pw + OFF_W3, 32, 14);
  conv_block<16, 32, 2>(sdy, bw, sd2, sh2);  // dh2 = W3^T dy (flipped) x relu'(h2)
  __syncthreads();
  weight_grad<32, 32>(sh1, sd2, pw + OFF_W2, 32, 32);
  conv_block<32, 32, 2>(sd2, bw + F3 / 4, sd1, sh1);  // dh1 = W2^T dh2 x relu'(h1)
  __syncthreads();
  weight_grad<16, 32>(sx, sd1, pw + OFF_W1, 15, 32);
}

// g[i] = sum_b partial[b][i] (fixed order)
__global__ void k_net_reduce(const float* __restrict__ partial, int nb, float* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNetParams) return;
  float s = 0.0f;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * kNetParams + i];
  g[i] = s;
}

// ------------------------------------------------------------ packing
// forward fragment: value j of lane = W[co = ct 16 + lane%16][ci = kb 16 + 4 (lane/16) + j][o]
// transposed:       value j of lane = W[co = kb 16 + 4 (lane/16) + j][ci = ct 16 + lane%16][26 - o]
__global__ void k_net_pack(const float* __restrict__ w, uint16_t* __restrict__ fw, uint16_t* __restrict__ bw) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int total_f = F1 + F2 + F3, total_b = F3 + F2;  // transposed: layer 3 (16->32), layer 2 (32->32)
  if (t < total_f) {
    int off = t, cip, cop, cin, cout, base;
    if (off < F1) { cip = 16; cop = 32; cin = 15; cout = 32; base = OFF_W1; }
    else if (off < F1 + F2) { off -= F1; cip = 32; cop = 32; cin = 32; cout = 32; base = OFF_W2; }
    else { off -= F1 + F2; cip = 32; cop = 16; cin = 32; cout = 14; base = OFF_W3; }
    const int KB = cip / 16, CT = cop / 16;
    int j = off % 4, lane = (off / 4) % 64, rest = off / 256;
    int ct = rest % CT, kb = (rest / CT) % KB, o = rest / (CT * KB);
    int co = ct * 16 + lane % 16, ci = kb * 16 + 4 * (lane / 16) + j;
    float v = (co < cout && ci < cin) ? w[base + ((int64_t)co * cin + ci) * 27 + o] : 0.0f;
    fw[t] = to_bf16(v);
  } else if (t < total_f + total_b) {
    int off = t - total_f, cip, cop, cin, cout, base;  // cip/cop of the transposed layer
    if (off < F3) { cip = 16; cop = 32; cin = 32; cout = 14; base = OFF_W3; }
    else { off -= F3; cip = 32; cop = 32; cin = 32; cout = 32; base = OFF_W2; }
    const int KB = cip / 16, CT = cop / 16;
    int j = off % 4, lane = (off / 4) % 64, rest = off / 256;
    int ct = rest % CT, kb = (rest / CT) % KB, o = rest / (CT * KB);
    int co = kb * 16 + 4 * (lane / 16) + j, ci = ct * 16 + lane % 16;  // forward-layer indices
    float v = (co < cout && ci < cin) ? w[base + ((int64_t)co * cin + ci) * 27 + (26 - o)] : 0.0f;
    bw[t - total_f] = to_bf16(v);
  }
}

// ------------------------------------------------------------ inputs / head
// One wave per sample (n, cell) of a Q2/P1 x DG(1) level, four samples per
// work group (a quarter of the work groups of one per sample).
template <typename T>
__global__ __launch_bounds__(256) void k_net_inputs(LevelArgs L, const T* __restrict__ r, const T* __restrict__ e,
                                                    int64_t first, int64_t count, uint16_t* __restrict__ x,
                                                    float* __restrict__ scale, float* __restrict__ mask,
                                                    float* __restrict__ tv, float* __restrict__ tp) {
  const int wave = threadIdx.x / 64;
  const int64_t sidx = (int64_t)blockIdx.x * 4 + wave;
  if (sidx >= count) return;  // (uniform over the wave; the work group has no barrier)
  const int64_t smp = first + sidx, ncell = n_cells(L);
  const int n = (int)(smp / ncell);
  const int64_t cell = smp - (int64_t)n * ncell;
  const int lane = threadIdx.x % 64, p = lane;
  int cc[3];
  cell_coords(L, cell, cc);
  bool fr = false;
  int64_t g = 0;
  if (p < 27) {
    int pi[3] = {p % 3, (p / 3) % 3, p / 9};
    int64_t st = 1;
    fr = true;
    for (int j = 0; j < 3; ++j) {
      int gj = cc[j] * L.q + pi[j];
      if (gj == 0 || gj == L.nn - 1) fr = false;
      g += gj * st;
      st *= L.nn;
    }
  }
  float vel[6] = {0, 0, 0, 0, 0, 0};
  float ssq = 0.0f;
  if (p < 27 && fr)
    for (int a = 0; a < 2; ++a)
      for (int comp = 0; comp < 3; ++comp) {
        float v = (float)r[(int64_t)n * L.slab + a * L.Mv + comp * L.nodes + g];
        vel[comp * 2 + a] = v;
        ssq += v * v;
      }
  float pres = 0.0f;
  if (lane < 8) {
    int a = lane / 4, l = lane % 4;
    pres = (float)r[(int64_t)n * L.slab + 2 * L.Mv + a * L.Mp + cell * L.C + l];
    ssq += pres * pres;
  }
  for (int off = 32; off > 0; off >>= 1) ssq += __shfl_xor(ssq, off, 64);
  const float s = sqrtf(ssq), inv = s > 0.0f ? 1.0f / s : 0.0f;
  float sp[8];  // the 8 pressure inputs, from lanes 0..7
#pragma unroll
  for (int c = 0; c < 8; ++c) sp[c] = __shfl(pres * inv, c, 64);
  uint16_t* xs = x + sidx * 512;
  if (p < 32) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float v = 0.0f;
      if (p < 27) {
        if (c < 6) v = vel[c] * inv;
        else if (c < 14) v = sp[c - 6];
        else if (c == 14) v = fr ? 0.0f : 1.0f;
      }
      xs[p * 16 + c] = to_bf16(v);
    }
  }
  if (p < 27) mask[sidx * 27 + p] = fr ? 0.0f : 1.0f;
  if (lane == 0) scale[sidx] = s;
  if (e) {
    if (p < 27)
      for (int a = 0; a < 2; ++a)
        for (int comp = 0; comp < 3; ++comp)
          tv[(sidx * 6 + comp * 2 + a) * 27 + p] =
              fr ? (float)e[(int64_t)n * L.slab + a * L.Mv + comp * L.nodes + g] * inv : 0.0f;
    if (lane < 8) {
      int a = lane / 4, l = lane % 4;
      tp[sidx * 8 + lane] = (float)e[(int64_t)n * L.slab + 2 * L.Mv + a * L.Mp + cell * L.C + l] * inv;
    }
  }
}

// velocity correction s_T * y (masked) into E (Vanka scratch layout), pressure
// added to x (assign: written to x, which then holds no values yet)
template <typename T>
__global__ __launch_bounds__(256) void k_net_correction(LevelArgs L, const float* __restrict__ y,
                                                        const float* __restrict__ scale,
                                                        const float* __restrict__ mask, int64_t first,
                                                        int64_t count, T* __restrict__ E, T* __restrict__ x,
                                                        int assign) {
  const int64_t sidx = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;  // one wave per sample
  if (sidx >= count) return;
  const int64_t smp = first + sidx, ncell = n_cells(L);
  const int n = (int)(smp / ncell);
  const int64_t cell = smp - (int64_t)n * ncell;
  const int lane = threadIdx.x % 64;
  const float s = scale[sidx];
  const float* ys = y + sidx * 512;
  if (lane < 27) {
    const float keep = 1.0f - mask[sidx * 27 + lane];
    for (int a = 0; a < 2; ++a)
      for (int comp = 0; comp < 3; ++comp)
        E[e_index(L, (int64_t)(n * 2 + a) * 3 + comp, cell, lane)] =
            (T)(s * keep * ys[lane * 16 + comp * 2 + a]);
  }
  if (lane < 8) {
    float m = 0.0f;
    for (int p = 0; p < 27; ++p) m += ys[p * 16 + 6 + lane];
    int a = lane / 4, l = lane % 4;
    T& xp = x[(int64_t)n * L.slab + 2 * L.Mv + a * L.Mp + cell * L.C + l];
    xp = (assign ? T(0) : xp) + (T)(s * m / 27.0f);
  }
}

// dy = 2 (head - t) through the head (unscaled; the 1/den factor is applied
// to the gradient), and the sums |head - t|^2, |t|^2 per block
__global__ __launch_bounds__(64) void k_net_loss(const float* __restrict__ y, const float* __restrict__ mask,
                                                 const float* __restrict__ tv, const float* __restrict__ tp,
                                                 int64_t count, uint16_t* __restrict__ dy, double* __restrict__ part) {
  const int64_t sidx = blockIdx.x;
  const int lane = threadIdx.x;
  const float* ys = y + sidx * 512;
  double se = 0.0, st = 0.0;
  float dp = 0.0f;
  if (lane < 8) {
    float m = 0.0f;
    for (int p = 0; p < 27; ++p) m += ys[p * 16 + 6 + lane];
    m /= 27.0f;
    float d = m - tp[sidx * 8 + lane];
    se += (double)d * d;
    st += (double)tp[sidx * 8 + lane] * tp[sidx * 8 + lane];
    dp = 2.0f * d / 27.0f;
  }
  __shared__ float sdp[8];
  if (lane < 8) sdp[lane] = dp;
  __syncthreads();
  if (lane < 32) {
    const int p = lane;
    const float keep = p < 27 ? 1.0f - mask[sidx * 27 + p] : 0.0f;
    for (int c = 0; c < 16; ++c) {
      float g = 0.0f;
      if (p < 27 && c < 6) {
        float t = tv[(sidx * 6 + c) * 27 + p];
        float d = ys[p * 16 + c] * keep - t;
        se += (double)d * d;
        st += (double)t * t;
        g = 2.0f * d * keep;
      } else if (p < 27 && c < 14) {
        g = sdp[c - 6];
      }
      dy[sidx * 512 + p * 16 + c] = to_bf16(g);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    se += __shfl_xor(se, off, 64);
    st += __shfl_xor(st, off, 64);
  }
  if (lane == 0) {
    part[2 * sidx] = se;
    part[2 * sidx + 1] = st;
  }
}

__global__ void k_net_loss_final(const double* __restrict__ part, int64_t count, double* __restrict__ red) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double se = 0.0, st = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    se += part[2 * i];
    st += part[2 * i + 1];
  }
  red[0] = se;
  red[1] = st;
}

__global__ void k_net_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, const double* __restrict__ red, float lr, float bc1,
                           float bc2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNetParams) return;
  const float den = red[1] > 0.0 ? (float)red[1] : 1.0f;
  const float gi = g[i] / den;
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

}  // namespace

// ========================================================= host wrappers
hipError_t net_pack(NetDev& N, hipStream_t s) {
  const int total = F1 + F2 + F3 + F3 + F2;
  k_net_pack<<<(total + 255) / 256, 256, 0, s>>>(N.w, N.fw, N.bw);
  return hipGetLastError();
}

template <typename T>
hipError_t net_inputs(const LevelArgs& L, NetDev& N, const T* r, const T* e, int64_t first, int64_t count,
                      hipStream_t s) {
  if (count > N.cap || L.d != 3 || L.Q != 3 || L.nt != 2) return hipErrorInvalidValue;
  k_net_inputs<T><<<(unsigned)((count + 3) / 4), 256, 0, s>>>(L, r, e, first, count, N.x, N.scale, N.mask, N.tv,
                                                               N.tp);
  return hipGetLastError();
}

hipError_t net_forward(NetDev& N, int64_t count, hipStream_t s, bool keep) {
  if (count > N.cap) return hipErrorInvalidValue;
  if (keep)
    k_net_fwd<<<(unsigned)((count + G - 1) / G), 256, 0, s>>>(N.x, reinterpret_cast<const bf16x4*>(N.fw), N.h1,
                                                              N.h2, N.y, count);
  else
    k_net_infer<<<(unsigned)((count + GI - 1) / GI), 256, 0, s>>>(N.x, reinterpret_cast<const bf16x4*>(N.fw), N.y,
                                                                  count);
  return hipGetLastError();
}

template <typename T>
hipError_t net_correction(const LevelArgs& L, NetDev& N, int64_t first, int64_t count, T* E, T* x, hipStream_t s,
                          bool assign) {
  k_net_correction<T><<<(unsigned)((count + 3) / 4), 256, 0, s>>>(L, N.y, N.scale, N.mask, first, count, E, x,
                                                                  assign ? 1 : 0);
  return hipGetLastError();
}

hipError_t net_loss(NetDev& N, int64_t count, hipStream_t s) {
  double* part = N.red + 2;
  k_net_loss<<<(unsigned)count, 64, 0, s>>>(N.y, N.mask, N.tv, N.tp, count, N.dy, part);
  k_net_loss_final<<<1, 64, 0, s>>>(part, count, N.red);
  return hipGetLastError();
}

hipError_t net_backward(NetDev& N, int64_t count, hipStream_t s) {
  const int64_t nb = (count + G - 1) / G;
  if (nb > N.pcap) return hipErrorInvalidValue;
  k_net_bwd<<<(unsigned)nb, 256, 0, s>>>(N.x, N.h1, N.h2, N.dy, reinterpret_cast<const bf16x4*>(N.bw), N.partial,
                                         count);
  k_net_reduce<<<(kNetParams + 255) / 256, 256, 0, s>>>(N.partial, (int)nb, N.g);
  return hipGetLastError();
}

hipError_t net_adam(NetDev& N, int t, float lr, hipStream_t s) {
  const float bc1 = 1.0f - powf(0.9f, (float)t), bc2 = 1.0f - powf(0.999f, (float)t);
  k_net_adam<<<(kNetParams + 255) / 256, 256, 0, s>>>(N.w, N.m, N.v, N.g, N.red, lr, bc1, bc2);
  return net_pack(N, s);
}

template hipError_t net_inputs<double>(const LevelArgs&, NetDev&, const double*, const double*, int64_t, int64_t,
                                       hipStream_t);
template hipError_t net_inputs<float>(const LevelArgs&, NetDev&, const float*, const float*, int64_t, int64_t,
                                      hipStream_t);
template hipError_t net_correction<double>(const LevelArgs&, NetDev&, int64_t, int64_t, double*, double*,
                                           hipStream_t, bool);
template hipError_t net_correction<float>(const LevelArgs&, NetDev&, int64_t, int64_t, float*, float*, hipStream_t,
                                          bool);

}  // namespace stmg
