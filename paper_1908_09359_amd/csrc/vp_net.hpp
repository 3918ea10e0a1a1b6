// Plaquette proposal network: parameter layout and the local evaluation used
// inside the learned sweep.
//
// Network f(S) (a proposal mechanism added on top of the sequential sampler of
// Sec. II.A Eq. (9); not in the paper): spins as +1 (s = 0) / -1 (s = 1) in
// one channel; conv3x3(1->32), ReLU, conv3x3(32->32), ReLU, conv3x3(32->32),
// ReLU, conv3x3(32->1); zero padding at the open boundary; each convolution is
// out[co][y][x] = b[co] + sum W[co][ci][ky][kx] in[ci][y+ky-1][x+kx-1].  The
// logit of plaquette (y, x) is the output at its top-left site.
//
// Flat parameters: W1[32][1][3][3] b1[32] W2[32][32][3][3] b2[32]
//                  W3[32][32][3][3] b3[32] W4[1][32][3][3] b4[1].
#pragma once

#include "vp_device.hpp"

namespace vp {

constexpr int NET_CH = 32;
constexpr int NET_OFF_W1 = 0;
constexpr int NET_OFF_B1 = NET_OFF_W1 + NET_CH * 9;
constexpr int NET_OFF_W2 = NET_OFF_B1 + NET_CH;
constexpr int NET_OFF_B2 = NET_OFF_W2 + NET_CH * NET_CH * 9;
constexpr int NET_OFF_W3 = NET_OFF_B2 + NET_CH;
constexpr int NET_OFF_B3 = NET_OFF_W3 + NET_CH * NET_CH * 9;
constexpr int NET_OFF_W4 = NET_OFF_B3 + NET_CH;
constexpr int NET_OFF_B4 = NET_OFF_W4 + NET_CH * 9;
constexpr int NET_NPARAM = NET_OFF_B4 + 1;

// LDS of one local evaluation (elements of T): 9x9 input, 7x7x32, 5x5x32 and
// 3x3x32 activations.
constexpr int NET_LOCAL_ELEMS = 81 + NET_CH * 49 + NET_CH * 25 + NET_CH * 9;
template <typename T>
constexpr size_t net_lds_bytes() { return sizeof(T) * NET_LOCAL_ELEMS; }

// The logit of plaquette (y, x) for the configuration sp (row-major Ly x Lx),
// with the four spins of that plaquette flipped when flip != 0.  Only the 9x9
// window the four layers see is evaluated; activations at positions outside
// the lattice are zero, as the zero padding of every layer requires.  All
// threads of the work-group call it; the result is returned to every thread.
template <typename T>
__device__ double net_logit(const T* __restrict__ W, const int8_t* sp, int Ly, int Lx, int y, int x, int flip,
                            char* lds) {
  T* in = reinterpret_cast<T*>(lds);  // [9][9]
  T* a1 = in + 81;                    // [32][7][7]
  T* a2 = a1 + NET_CH * 49;           // [32][5][5]
  T* a3 = a2 + NET_CH * 25;           // [32][3][3]
  const int tid = threadIdx.x;
  for (int i = tid; i < 81; i += WG) {
    const int yy = y - 4 + i / 9, xx = x - 4 + i % 9;
    T v = T(0);
    if (yy >= 0 && yy < Ly && xx >= 0 && xx < Lx) {
      int s = sp[yy * Lx + xx];
      if (flip && (yy == y || yy == y + 1) && (xx == x || xx == x + 1)) s ^= 1;
      v = s ? T(-1) : T(1);
    }
    in[i] = v;
  }
  __syncthreads();
  // layer 1 on the 7x7 window centred at (y, x); input window offset 1
  for (int i = tid; i < NET_CH * 49; i += WG) {
    const int co = i / 49, p = i % 49, py = p / 7, px = p % 7;
    const int yy = y - 3 + py, xx = x - 3 + px;
    T v = T(0);
    if (yy >= 0 && yy < Ly && xx >= 0 && xx < Lx) {
      T acc = W[NET_OFF_B1 + co];
#pragma unroll
      for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) acc += W[NET_OFF_W1 + co * 9 + ky * 3 + kx] * in[(py + ky) * 9 + px + kx];
      v = acc > T(0) ? acc : T(0);
    }
    a1[i] = v;
  }
  __syncthreads();
  // layer 2 on the 5x5 window
  for (int i = tid; i < NET_CH * 25; i += WG) {
    const int co = i / 25, p = i % 25, py = p / 5, px = p % 5;
    const int yy = y - 2 + py, xx = x - 2 + px;
    T v = T(0);
    if (yy >= 0 && yy < Ly && xx >= 0 && xx < Lx) {
      T acc = W[NET_OFF_B2 + co];
      const T* w = W + NET_OFF_W2 + co * NET_CH * 9;
      for (int ci = 0; ci < NET_CH; ++ci)
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
          for (int kx = 0; kx < 3; ++kx) acc += w[ci * 9 + ky * 3 + kx] * a1[ci * 49 + (py + ky) * 7 + px + kx];
      v = acc > T(0) ? acc : T(0);
    }
    a2[i] = v;
  }
  __syncthreads();
  // layer 3 on the 3x3 window
  for (int i = tid; i < NET_CH * 9; i += WG) {
    const int co = i / 9, p = i % 9, py = p / 3, px = p % 3;
    const int yy = y - 1 + py, xx = x - 1 + px;
    T v = T(0);
    if (yy >= 0 && yy < Ly && xx >= 0 && xx < Lx) {
      T acc = W[NET_OFF_B3 + co];
      const T* w = W + NET_OFF_W3 + co * NET_CH * 9;
      for (int ci = 0; ci < NET_CH; ++ci)
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
          for (int kx = 0; kx < 3; ++kx) acc += w[ci * 9 + ky * 3 + kx] * a2[ci * 25 + (py + ky) * 5 + px + kx];
      v = acc > T(0) ? acc : T(0);
    }
    a3[i] = v;
  }
  __syncthreads();
  // layer 4 at (y, x): 288 products, reduced over the work-group
  double part = 0.0;
  for (int i = tid; i < NET_CH * 9; i += WG) part += (double)(W[NET_OFF_W4 + i] * a3[i]);
  const double z = wg_sum(part) + (double)W[NET_OFF_B4];
  return z;
}

// Packed copy of the parameters for bf16 inference (net_pack_bf16): float
// biases b1[32] b2[32] b3[32] b4 (padded to NBF_FLOATS floats), then bf16
// weights W1[co][tap], W2[tap][co][ci], W3[tap][co][ci], W4[tap][ci]
// (tap = 3 ky + kx), each rounded to nearest bf16 (ties to even).  The W2 and
// W3 rows of 32 input channels start on 16-byte boundaries.
constexpr int NBF_FLOATS = 100;
constexpr int NBF_W1 = 0;
constexpr int NBF_W2 = NBF_W1 + NET_CH * 9;
constexpr int NBF_W3 = NBF_W2 + 9 * NET_CH * NET_CH;
constexpr int NBF_W4 = NBF_W3 + 9 * NET_CH * NET_CH;
constexpr int NBF_N = NBF_W4 + 9 * NET_CH;
constexpr size_t NET_BF_BYTES = sizeof(float) * NBF_FLOATS + 2 * NBF_N;
static_assert((sizeof(float) * NBF_FLOATS) % 16 == 0 && (2 * NBF_W2) % 16 == 0 && (2 * NBF_W3) % 16 == 0,
              "bf16 weight rows on 16-byte boundaries");

// LDS of one bf16 local evaluation: the 9x9 input (float), layer-1 and layer-2
// activations (bf16, [position][channel], rows of NBF_ROW for 16-byte
// aligned 8-channel reads), layer-3 activations (float).
constexpr int NBF_ROW = NET_CH + 8;
constexpr size_t NBF_IN = 336, NBF_A1 = NBF_IN + 2 * 49 * NBF_ROW, NBF_A2 = NBF_A1 + 2 * 25 * NBF_ROW;
constexpr size_t net_bf_lds_bytes() { return NBF_A2 + sizeof(float) * 9 * NET_CH; }

// The logit of plaquette (y, x) as net_logit computes it, in bf16 inference:
// weights and ReLU outputs in bf16, float32 accumulation.  Layer 1 (one input
// channel) on the vector ALU; layers 2 and 3 as implicit GEMMs on the bf16
// MFMA (16x16x32): rows are the output positions of the 5x5 (3x3) window,
// columns the 32 output channels, and each of the 9 k-steps is one tap (ky,
// kx) over the 32 input channels; layer 4 (288 products, exact in float32) is
// summed over the work-group in float64.  Activations at positions outside the
// lattice are zero.  All threads of the work-group call it.
__device__ inline double net_logit_bf16(const char* __restrict__ P, const int8_t* sp, int Ly, int Lx, int y, int x,
                                        int flip, char* lds) {
  const float* bias = reinterpret_cast<const float*>(P);
  const __bf16* Wb = reinterpret_cast<const __bf16*>(P + sizeof(float) * NBF_FLOATS);
  float* in = reinterpret_cast<float*>(lds);
  __bf16* a1 = reinterpret_cast<__bf16*>(lds + NBF_IN);
  __bf16* a2 = reinterpret_cast<__bf16*>(lds + NBF_A1);
  float* a3 = reinterpret_cast<float*>(lds + NBF_A2);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < 81; i += WG) {
    const int yy = y - 4 + i / 9, xx = x - 4 + i % 9;
    float v = 0.0f;
    if (yy >= 0 && yy < Ly && xx >= 0 && xx < Lx) {
      int s = sp[yy * Lx + xx];
      if (flip && (yy == y || yy == y + 1) && (xx == x || xx == x + 1)) s ^= 1;
      v = s ? -1.0f : 1.0f;
    }
    in[i] = v;
  }
  __syncthreads();
  // layer 1 on the 7x7 window centred at (y, x)
  for (int i = tid; i < NET_CH * 49; i += WG) {
    const int co = i / 49, p = i % 49, py = p / 7, px = p % 7;
    const int yy = y - 3 + py, xx = x - 3 + px;
    float v = 0.0f;
    if (yy >= 0 && yy < Ly && xx >= 0 && xx < Lx) {
      float acc = bias[co];
#pragma unroll
      for (int t = 0; t < 9; ++t) acc += (float)Wb[NBF_W1 + co * 9 + t] * in[(py + t / 3) * 9 + px + t % 3];
      v = fmaxf(acc, 0.0f);
    }
    a1[p * NBF_ROW + co] = (__bf16)v;
  }
  __syncthreads();
  const int kq = (lane >> 4) * 8;
  const v8bf_g zero8 = {};
  // layer 2 on the 5x5 window: wave w computes positions 16 (w >> 1) .. +15, channels 16 (w & 1) .. +15
  {
    const int p = 16 * (wave >> 1) + (lane & 15), co = 16 * (wave & 1) + (lane & 15);
    const int py = p / 5, px = p % 5;
    v4f_g acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const v8bf_g a =
          p < 25 ? *reinterpret_cast<const v8bf_g*>(a1 + ((py + t / 3) * 7 + px + t % 3) * NBF_ROW + kq) : zero8;
      const v8bf_g b = *reinterpret_cast<const v8bf_g*>(Wb + NBF_W2 + (t * NET_CH + co) * NET_CH + kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 16 * (wave >> 1) + 4 * (lane >> 4) + r;
      if (q < 25) {
        const int yy = y - 2 + q / 5, xx = x - 2 + q % 5;
        const bool inside = yy >= 0 && yy < Ly && xx >= 0 && xx < Lx;
        a2[q * NBF_ROW + co] = (__bf16)(inside ? fmaxf(acc[r] + bias[NET_CH + co], 0.0f) : 0.0f);
      }
    }
  }
  __syncthreads();
  // layer 3 on the 3x3 window: waves 0 and 1, channels 16 w .. +15
  if (wave < 2) {
    const int p = lane & 15, co = 16 * wave + (lane & 15);
    const int py = p / 3, px = p % 3;
    v4f_g acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const v8bf_g a =
          p < 9 ? *reinterpret_cast<const v8bf_g*>(a2 + ((py + t / 3) * 5 + px + t % 3) * NBF_ROW + kq) : zero8;
      const v8bf_g b = *reinterpret_cast<const v8bf_g*>(Wb + NBF_W3 + (t * NET_CH + co) * NET_CH + kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * (lane >> 4) + r;
      if (q < 9) {
        const int yy = y - 1 + q / 3, xx = x - 1 + q % 3;
        const bool inside = yy >= 0 && yy < Ly && xx >= 0 && xx < Lx;
        a3[q * NET_CH + co] = (float)(__bf16)(inside ? fmaxf(acc[r] + bias[2 * NET_CH + co], 0.0f) : 0.0f);
      }
    }
  }
  __syncthreads();
  // layer 4 at (y, x): tap t of the 3x3 window is the window position t
  double part = 0.0;
  for (int i = tid; i < NET_CH * 9; i += WG) part += (double)((float)Wb[NBF_W4 + i] * a3[i]);
  return wg_sum(part) + (double)bias[3 * NET_CH];
}

__device__ inline double net_sigmoid(double z) {
  if (z >= 0.0) return 1.0 / (1.0 + exp(-z));
  const double e = exp(z);
  return e / (1.0 + e);
}

}  // namespace vp
