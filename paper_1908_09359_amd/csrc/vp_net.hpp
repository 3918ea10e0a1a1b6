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

__device__ inline double net_sigmoid(double z) {
  if (z >= 0.0) return 1.0 / (1.0 + exp(-z));
  const double e = exp(z);
  return e / (1.0 + e);
}

}  // namespace vp
