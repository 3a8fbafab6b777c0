// Learned correction after a Vanka sweep: a 3-layer 3x3x3 convolutional
// network on the cell-local residual of the Q2/P1 x DG(1) element, BF16
// operands on the matrix cores with FP32 accumulation.  Forward (inference
// and training), backward (data and weight gradients) and Adam.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace stmg {

// Network sizes (channels padded to multiples of 16 on the device).
constexpr int kNetCin = 15, kNetHid = 32, kNetCout = 14;
constexpr int kNetParams = kNetHid * kNetCin * 27 + kNetHid * kNetHid * 27 + kNetCout * kNetHid * 27;
// Weights in the host/ABI order: W1 (32 x 15 x 27), W2 (32 x 32 x 27), W3 (14 x 32 x 27),
// each [c_out][c_in][offset], offset o = (dx+1) + 3 (dy+1) + 9 (dz+1).

// Device buffers of one network (weights, optimiser state, fragments, workspace).
struct NetDev {
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // FP32 master weights, Adam moments, gradient
  uint16_t *fw = nullptr;   // BF16 B-operand fragments of the forward layers
  uint16_t *bw = nullptr;   // BF16 fragments of the transposed/flipped layers (data gradients)
  int64_t cap = 0;          // samples the workspace holds
  uint16_t *x = nullptr, *h1 = nullptr, *h2 = nullptr;  // activations [sample][32][C]
  float* y = nullptr;       // raw output [sample][32][16]
  uint16_t *dy = nullptr, *dh2 = nullptr, *dh1 = nullptr;
  float* scale = nullptr;   // s_T per sample
  float* mask = nullptr;    // Dirichlet mask per sample [27]
  float* tv = nullptr;      // targets [sample][6][27] and [sample][8] (normalised)
  float* tp = nullptr;
  float* partial = nullptr; // per-workgroup weight-gradient partials
  double* red = nullptr;    // loss reduction scratch
  int64_t pcap = 0;         // workgroups the partial buffer holds
};

// Rebuild the BF16 fragments from the FP32 master weights.
hipError_t net_pack(NetDev& N, hipStream_t s);

// Build normalised inputs for samples (cell, n) of a level vector v (T) and
// optionally targets from an error vector e (T):  samples are
// [first, first + count) in the order n-major, then cell.
template <typename T>
hipError_t net_inputs(const LevelArgs& L, NetDev& N, const T* r, const T* e, int64_t first, int64_t count,
                      hipStream_t s);

// Forward pass over `count` samples held in the workspace; keep: also store
// the hidden activations (for a backward pass), else inference only.
hipError_t net_forward(NetDev& N, int64_t count, hipStream_t s, bool keep);

// Correction head: cell-local velocity corrections (times s_T) into E
// (the Vanka scratch layout) and pressure corrections added to x (assign:
// written to x, whose pressure entries then need no initial values).
template <typename T>
hipError_t net_correction(const LevelArgs& L, NetDev& N, int64_t first, int64_t count, T* E, T* x, hipStream_t s,
                          bool assign = false);

// Loss of the head against the targets; writes dL/dy into the workspace and
// accumulates sum |head - t|^2 and sum |t|^2 into red[0], red[1].
hipError_t net_loss(NetDev& N, int64_t count, hipStream_t s);

// Backward pass: weight gradient into N.g (overwritten), given dy.
// The gradient is of sum |head - t|^2 / den with den = red[1] read on the device.
hipError_t net_backward(NetDev& N, int64_t count, hipStream_t s);

// Adam step on the master weights (step t >= 1), then re-pack.
hipError_t net_adam(NetDev& N, int t, float lr, hipStream_t s);

}  // namespace stmg
