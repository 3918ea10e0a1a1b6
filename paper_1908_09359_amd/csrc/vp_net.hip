// Batched float32 kernels of the plaquette proposal network: forward pass,
// binary cross-entropy against the acceptance target min(1, R), reverse-mode
// gradient and the Adam step.  Layout of activations: [n][channels][Ly][Lx].
// Every reduction runs in a fixed order (no atomics), so training is
// reproducible run to run.
#include "vp_device.hpp"
#include "vp_kernels.hpp"
#include "vp_net.hpp"

#include <math.h>

#include <algorithm>
#include <mutex>

namespace vp {

// Activation scratch of the allocation-free forward pass
// (vp_proposal_forward_noalloc): a fixed array in device memory, one copy per
// GPU, held until the process ends.  Host code never passes this name to a
// kernel: on the host it is only a stand-in, and the device address of each
// GPU's copy is looked up once (net_scratch_setup) and used from then on.
static __device__ __align__(256) float scratch[NET_SCRATCH_FLOATS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t net_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<float*>(ptr);
  return hipSuccess;
}

float* net_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

namespace {

__global__ void k_net_input(const int8_t* __restrict__ spins, int64_t total, float* __restrict__ x) {
  for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < total; i += (int64_t)gridDim.x * WG)
    x[i] = spins[i] ? -1.0f : 1.0f;
}

// The 3x3 convolutions of training and of the batched forward pass as
// implicit GEMMs on the fp32 MFMA (16x16x4, float32 accumulation).  A
// work-group takes 64 rows of the batch's positions (b, y, x); wave w owns rows
// 16 w .. 16 w + 15 against every 16-column tile.  The contraction index k
// runs over (tap, channel), tap = 3 ky + kx, padded to a multiple of 4; the
// weight matrix is staged in LDS with rows of KP + 1 floats (the 16 columns a
// step reads then fall in distinct banks).  Positions outside the lattice read
// zero (the zero padding of every layer).
constexpr int CONV_ROWS = 64;

template <int CI, int CO>
struct ConvShape {
  static constexpr int K = 9 * CI, KP = (K + 3) / 4 * 4, NT = (CO + 15) / 16, LD = KP + 1;
};

// out[b][co][y][x] = bias[co] + sum W[co][ci][ky][kx] in[b][ci][y+ky-1][x+kx-1], ReLU if RELU.
template <int CI, int CO, bool RELU>
__global__ void __launch_bounds__(WG) k_conv_fwd(const float* __restrict__ in, const float* __restrict__ W,
                                                 const float* __restrict__ bias, float* __restrict__ out, int n, int H,
                                                 int Wd) {
  using S = ConvShape<CI, CO>;
  __shared__ float Wl[S::NT * 16 * S::LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < S::NT * 16 * S::KP; e += WG) {
    const int co = e / S::KP, k = e % S::KP, tap = k / CI, ci = k % CI;
    Wl[co * S::LD + k] = (co < CO && k < S::K) ? W[(co * CI + ci) * 9 + tap] : 0.0f;
  }
  __syncthreads();
  const int HW = H * Wd;
  const int64_t rows = (int64_t)n * HW;
  const int64_t r = (int64_t)blockIdx.x * CONV_ROWS + 16 * wave + (lane & 15);
  const bool valid = r < rows;
  const int64_t b = valid ? r / HW : 0;
  const int p = valid ? (int)(r % HW) : 0, y = p / Wd, x = p % Wd;
  v4f_g acc[S::NT];
#pragma unroll
  for (int t = 0; t < S::NT; ++t) acc[t] = v4f_g{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < S::KP; k0 += 4) {
    const int k = k0 + (lane >> 4), tap = k / CI, ci = k % CI;
    const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
    const float a = (valid && k < S::K && yy >= 0 && yy < H && xx >= 0 && xx < Wd)
                        ? in[(b * CI + ci) * HW + yy * Wd + xx] : 0.0f;
#pragma unroll
    for (int t = 0; t < S::NT; ++t) acc[t] = mfma4(a, Wl[(16 * t + (lane & 15)) * S::LD + k], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < S::NT; ++t) {
    const int co = 16 * t + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t rr = (int64_t)blockIdx.x * CONV_ROWS + 16 * wave + mfma4_row(0.0f, lane, q);
      if (co < CO && rr < rows) {
        const float v = acc[t][q] + bias[co];
        out[((rr / HW) * CO + co) * HW + rr % HW] = RELU ? fmaxf(v, 0.0f) : v;
      }
    }
  }
}

// Per configuration (one work-group each): BCE sum and count over its movable
// plaquettes, and dz = sigmoid(z) - a at their top-left sites (0 elsewhere);
// a = min(1, rho^2) from the plaquette-flip ratio rho.
__global__ void k_plaq_loss(const float* __restrict__ z, const int8_t* __restrict__ spins,
                            const double* __restrict__ ratios, int H, int Wd, float* __restrict__ dz,
                            double* __restrict__ part_loss, int* __restrict__ part_cnt) {
  const int64_t b = blockIdx.x;
  const int HW = H * Wd, P = (H - 1) * (Wd - 1);
  const int8_t* sp = spins + b * HW;
  double lsum = 0.0;
  int cnt = 0;
  for (int i = threadIdx.x; i < HW; i += WG) {
    const int y = i / Wd, x = i % Wd;
    float g = 0.0f;
    if (y < H - 1 && x < Wd - 1 && sp[i] + sp[i + 1] + sp[i + Wd] + sp[i + Wd + 1] == 2) {
      const double rho = ratios[b * P + y * (Wd - 1) + x];
      const double a = fmin(1.0, rho * rho);
      const double zz = (double)z[b * HW + i];
      lsum += fmax(zz, 0.0) - zz * a + log1p(exp(-fabs(zz)));
      g = (float)(net_sigmoid(zz) - a);
      cnt += 1;
    }
    dz[b * HW + i] = g;
  }
  lsum = wg_sum(lsum);
  const double c = wg_sum((double)cnt);
  if (threadIdx.x == 0) {
    part_loss[b] = lsum;
    part_cnt[b] = (int)c;
  }
}

// scal[0] = total loss / count, scal[1] = 1 / count (one work-group).
__global__ void k_loss_total(const double* __restrict__ part_loss, const int* __restrict__ part_cnt, int n,
                             double* __restrict__ scal) {
  double l = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n; i += WG) {
    l += part_loss[i];
    c += part_cnt[i];
  }
  l = wg_sum(l);
  c = wg_sum(c);
  if (threadIdx.x == 0) {
    scal[0] = c > 0 ? l / c : 0.0;
    scal[1] = c > 0 ? 1.0 / c : 0.0;
  }
}

__global__ void k_scale(float* __restrict__ v, int64_t n, const double* __restrict__ scal) {
  const float f = (float)scal[1];
  for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) v[i] *= f;
}

// din[b][ci][y][x] = [act(b,ci,y,x) > 0] sum_{co,ky,kx} W[co][ci][ky][kx] dout[b][co][y-ky+1][x-kx+1],
// the same implicit GEMM with k over (tap, co) and the transposed weights in LDS.
template <int CO, int CI>
__global__ void __launch_bounds__(WG) k_conv_bwd_data(const float* __restrict__ dout, const float* __restrict__ W,
                                                      const float* __restrict__ act, float* __restrict__ din, int n,
                                                      int H, int Wd) {
  using S = ConvShape<CO, CI>;  // contraction over (tap, co), columns ci
  __shared__ float Wl[S::NT * 16 * S::LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < S::NT * 16 * S::KP; e += WG) {
    const int ci = e / S::KP, k = e % S::KP, tap = k / CO, co = k % CO;
    Wl[ci * S::LD + k] = (ci < CI && k < S::K) ? W[(co * CI + ci) * 9 + tap] : 0.0f;
  }
  __syncthreads();
  const int HW = H * Wd;
  const int64_t rows = (int64_t)n * HW;
  const int64_t r = (int64_t)blockIdx.x * CONV_ROWS + 16 * wave + (lane & 15);
  const bool valid = r < rows;
  const int64_t b = valid ? r / HW : 0;
  const int p = valid ? (int)(r % HW) : 0, y = p / Wd, x = p % Wd;
  v4f_g acc[S::NT];
#pragma unroll
  for (int t = 0; t < S::NT; ++t) acc[t] = v4f_g{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < S::KP; k0 += 4) {
    const int k = k0 + (lane >> 4), tap = k / CO, co = k % CO;
    const int yy = y - tap / 3 + 1, xx = x - tap % 3 + 1;
    const float a = (valid && k < S::K && yy >= 0 && yy < H && xx >= 0 && xx < Wd)
                        ? dout[(b * CO + co) * HW + yy * Wd + xx] : 0.0f;
#pragma unroll
    for (int t = 0; t < S::NT; ++t) acc[t] = mfma4(a, Wl[(16 * t + (lane & 15)) * S::LD + k], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < S::NT; ++t) {
    const int ci = 16 * t + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t rr = (int64_t)blockIdx.x * CONV_ROWS + 16 * wave + mfma4_row(0.0f, lane, q);
      if (ci < CI && rr < rows) {
        const int64_t o = ((rr / HW) * CI + ci) * HW + rr % HW;
        din[o] = act[o] > 0.0f ? acc[t][q] : 0.0f;
      }
    }
  }
}

// Weight gradient gW[co][(ci, tap)] = sum over positions of dout[b][co][p] in[b][ci][p + tap offset]:
// an implicit GEMM (rows co, columns (ci, tap)) whose contraction runs over the
// batch's positions, split into chunks of CONV_WCHUNK positions, one
// work-group per chunk writing its partial product; wave w owns tiles
// w, w + 4, ... of the (CO / 16) x (9 CI / 16) output tiles.
constexpr int CONV_WCHUNK = 256;

template <int CO, int CI>
__global__ void __launch_bounds__(WG) k_conv_wgrad_part(const float* __restrict__ dout, const float* __restrict__ in,
                                                        float* __restrict__ part, int n, int H, int Wd) {
  constexpr int MT = (CO + 15) / 16, NC = 9 * CI, NTN = (NC + 15) / 16, NTILE = MT * NTN;
  constexpr int TW = (NTILE + 3) / 4;  // tiles per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int HW = H * Wd;
  const int64_t rows = (int64_t)n * HW, r0 = (int64_t)blockIdx.x * CONV_WCHUNK;
  v4f_g acc[TW];
#pragma unroll
  for (int j = 0; j < TW; ++j) acc[j] = v4f_g{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < CONV_WCHUNK; k0 += 4) {
    const int64_t r = r0 + k0 + (lane >> 4);
    const bool valid = r < rows;
    const int64_t b = valid ? r / HW : 0;
    const int p = valid ? (int)(r % HW) : 0, y = p / Wd, x = p % Wd;
#pragma unroll
    for (int j = 0; j < TW; ++j) {
      const int tile = wave + 4 * j;
      if (tile < NTILE) {  // uniform over the wavefront
        const int mt = tile / NTN, nt = tile % NTN;
        const int co = 16 * mt + (lane & 15), col = 16 * nt + (lane & 15);
        const float a = (valid && co < CO) ? dout[(b * CO + co) * HW + p] : 0.0f;
        const int ci = col / 9, tap = col % 9, yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        const float bv = (valid && col < NC && yy >= 0 && yy < H && xx >= 0 && xx < Wd)
                             ? in[(b * CI + ci) * HW + yy * Wd + xx] : 0.0f;
        acc[j] = mfma4(a, bv, acc[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < TW; ++j) {
    const int tile = wave + 4 * j;
    if (tile < NTILE) {
      const int mt = tile / NTN, nt = tile % NTN, col = 16 * nt + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int co = 16 * mt + mfma4_row(0.0f, lane, q);
        if (co < CO && col < NC) part[((int64_t)blockIdx.x * CO + co) * NC + col] = acc[j][q];
      }
    }
  }
}

// gW[j] = sum over the chunks of part[c][j] (float64, chunk order); gb[co] =
// sum over positions of dout[b][co][p] (float64, fixed order; one work-group per co).
__global__ void k_conv_wgrad_sum(const float* __restrict__ part, int nchunk, int nw, float* __restrict__ gW) {
  for (int j = blockIdx.x * WG + threadIdx.x; j < nw; j += gridDim.x * WG) {
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += (double)part[(int64_t)c * nw + j];
    gW[j] = (float)acc;
  }
}

__global__ void k_conv_bgrad(const float* __restrict__ dout, int Co, float* __restrict__ gb, int n, int H, int Wd) {
  const int co = blockIdx.x;
  const int64_t HW = (int64_t)H * Wd, total = (int64_t)n * HW;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < total; i += WG) acc += (double)dout[((i / HW) * Co + co) * HW + i % HW];
  acc = wg_sum(acc);
  if (threadIdx.x == 0) gb[co] = (float)acc;
}

// Adam (Kingma & Ba, 2015) with bias correction; t is the 1-based step.
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, int t) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_gather_batch(const int8_t* __restrict__ spins, const double* __restrict__ ratios,
                               const int32_t* __restrict__ idx, int nb, int HW, int P, int8_t* __restrict__ sb,
                               double* __restrict__ rb) {
  const int b = blockIdx.x;
  if (b >= nb) return;
  const int64_t src = idx[b];
  for (int i = threadIdx.x; i < HW; i += WG) sb[(int64_t)b * HW + i] = spins[src * HW + i];
  for (int i = threadIdx.x; i < P; i += WG) rb[(int64_t)b * P + i] = ratios[src * P + i];
}

template <typename T>
__global__ void k_cast_params(const float* __restrict__ src, T* __restrict__ dst, int n) {
  for (int i = blockIdx.x * WG + threadIdx.x; i < n; i += gridDim.x * WG) dst[i] = (T)src[i];
}

unsigned grid_for(int64_t total) { return (unsigned)std::min<int64_t>((total + WG - 1) / WG, 65536); }

// The packed bf16 copy (layout in vp_net.hpp): element i of the bf16 region,
// then the biases.
__global__ void k_pack_bf16(const float* __restrict__ th, char* __restrict__ out) {
  __bf16* w = reinterpret_cast<__bf16*>(out + sizeof(float) * NBF_FLOATS);
  float* b = reinterpret_cast<float*>(out);
  for (int i = blockIdx.x * WG + threadIdx.x; i < NBF_N; i += gridDim.x * WG) {
    float v;
    if (i < NBF_W2) {  // W1[co][tap]
      v = th[NET_OFF_W1 + i];
    } else if (i < NBF_W4) {  // W2 / W3 [tap][co][ci] <- W[co][ci][tap]
      const int j = i < NBF_W3 ? i - NBF_W2 : i - NBF_W3;
      const int t = j / (NET_CH * NET_CH), co = (j / NET_CH) % NET_CH, ci = j % NET_CH;
      v = th[(i < NBF_W3 ? NET_OFF_W2 : NET_OFF_W3) + (co * NET_CH + ci) * 9 + t];
    } else {  // W4[tap][ci] <- W4[0][ci][tap]
      const int j = i - NBF_W4, t = j / NET_CH, ci = j % NET_CH;
      v = th[NET_OFF_W4 + ci * 9 + t];
    }
    w[i] = (__bf16)v;
  }
  for (int i = blockIdx.x * WG + threadIdx.x; i < NBF_FLOATS; i += gridDim.x * WG)
    b[i] = i < NET_CH ? th[NET_OFF_B1 + i]
           : i < 2 * NET_CH ? th[NET_OFF_B2 + i - NET_CH]
           : i < 3 * NET_CH ? th[NET_OFF_B3 + i - 2 * NET_CH]
           : i == 3 * NET_CH ? th[NET_OFF_B4] : 0.0f;
}

// The logits of every plaquette of n configurations as the learned sweep
// evaluates them (one work-group per configuration): bf16 inference from the
// packed copy, or the working-precision evaluation from W.
template <typename T, bool BF16>
__global__ void __launch_bounds__(WG) k_net_local(const T* __restrict__ W, const char* __restrict__ Pb,
                                                  const int8_t* __restrict__ spins, int H, int Wd, int flip,
                                                  double* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) char lds[BF16 ? net_bf_lds_bytes() : net_lds_bytes<T>()];
  const int n = blockIdx.x, P = (H - 1) * (Wd - 1);
  const int8_t* sp = spins + (int64_t)n * H * Wd;
  for (int q = 0; q < P; ++q) {
    const int y = q / (Wd - 1), x = q % (Wd - 1);
    double z;
    if constexpr (BF16) z = net_logit_bf16(Pb, sp, H, Wd, y, x, flip, lds);
    else z = net_logit<T>(W, sp, H, Wd, y, x, flip, lds);
    if (threadIdx.x == 0) out[(int64_t)n * P + q] = z;
    __syncthreads();
  }
}

}  // namespace

size_t net_forward_floats(int n, int H, int Wd) {
  // x, a1, a2, a3: what net_forward reads and writes besides its output
  return (size_t)n * H * Wd * (1 + 3 * NET_CH);
}

static size_t wgrad_chunks(int n, int H, int Wd) { return ((size_t)n * H * Wd + CONV_WCHUNK - 1) / CONV_WCHUNK; }

size_t net_work_floats(int n, int H, int Wd) {
  const size_t HW = (size_t)H * Wd;
  // x, a1, a2, a3, z, d3, d2, d1 (dz shares z's shape), then the weight-gradient partials
  return (size_t)n * HW * (1 + 3 * NET_CH + 1 + 1 + 3 * NET_CH) + wgrad_chunks(n, H, Wd) * NET_CH * NET_CH * 9;
}

template <int CO, int CI>
static void wgrad(const float* dout, const float* in, float* part, float* gW, float* gb, int n, int H, int Wd,
                  hipStream_t s) {
  const int nchunk = (int)wgrad_chunks(n, H, Wd), nw = CO * CI * 9;
  hipLaunchKernelGGL((k_conv_wgrad_part<CO, CI>), dim3(nchunk), dim3(WG), 0, s, dout, in, part, n, H, Wd);
  hipLaunchKernelGGL(k_conv_wgrad_sum, dim3(grid_for(nw)), dim3(WG), 0, s, part, nchunk, nw, gW);
  hipLaunchKernelGGL(k_conv_bgrad, dim3(CO), dim3(WG), 0, s, dout, CO, gb, n, H, Wd);
}

static unsigned conv_grid(int n, int H, int Wd) {
  return (unsigned)(((int64_t)n * H * Wd + CONV_ROWS - 1) / CONV_ROWS);
}

void net_forward(const float* th, const int8_t* spins, int n, int H, int Wd, float* work, float* logits,
                 hipStream_t s) {
  const int64_t HW = (int64_t)H * Wd;
  float* x = work;
  float* a1 = x + n * HW;
  float* a2 = a1 + n * NET_CH * HW;
  float* a3 = a2 + n * NET_CH * HW;
  const unsigned g = conv_grid(n, H, Wd);
  hipLaunchKernelGGL(k_net_input, dim3(grid_for(n * HW)), dim3(WG), 0, s, spins, n * HW, x);
  hipLaunchKernelGGL((k_conv_fwd<1, NET_CH, true>), dim3(g), dim3(WG), 0, s, x, th + NET_OFF_W1, th + NET_OFF_B1, a1,
                     n, H, Wd);
  hipLaunchKernelGGL((k_conv_fwd<NET_CH, NET_CH, true>), dim3(g), dim3(WG), 0, s, a1, th + NET_OFF_W2,
                     th + NET_OFF_B2, a2, n, H, Wd);
  hipLaunchKernelGGL((k_conv_fwd<NET_CH, NET_CH, true>), dim3(g), dim3(WG), 0, s, a2, th + NET_OFF_W3,
                     th + NET_OFF_B3, a3, n, H, Wd);
  hipLaunchKernelGGL((k_conv_fwd<NET_CH, 1, false>), dim3(g), dim3(WG), 0, s, a3, th + NET_OFF_W4, th + NET_OFF_B4,
                     logits, n, H, Wd);
}

void net_loss_grad(const float* th, const int8_t* spins, const double* ratios, int n, int H, int Wd, float* work,
                   double* part, int* cnt, double* scal, float* grad, hipStream_t s) {
  const int64_t HW = (int64_t)H * Wd;
  float* x = work;
  float* a1 = x + n * HW;
  float* a2 = a1 + n * NET_CH * HW;
  float* a3 = a2 + n * NET_CH * HW;
  float* z = a3 + n * NET_CH * HW;
  float* dz = z + n * HW;
  float* d3 = dz + n * HW;
  float* d2 = d3 + n * NET_CH * HW;
  float* d1 = d2 + n * NET_CH * HW;
  net_forward(th, spins, n, H, Wd, work, z, s);
  hipLaunchKernelGGL(k_plaq_loss, dim3(n), dim3(WG), 0, s, z, spins, ratios, H, Wd, dz, part, cnt);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(WG), 0, s, part, cnt, n, scal);
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n * HW)), dim3(WG), 0, s, dz, n * HW, (const double*)scal);
  float* wpart = d1 + n * NET_CH * HW;
  const unsigned g = conv_grid(n, H, Wd);
  // layer 4
  wgrad<1, NET_CH>(dz, a3, wpart, grad + NET_OFF_W4, grad + NET_OFF_B4, n, H, Wd, s);
  hipLaunchKernelGGL((k_conv_bwd_data<1, NET_CH>), dim3(g), dim3(WG), 0, s, dz, th + NET_OFF_W4, a3, d3, n, H, Wd);
  // layer 3
  wgrad<NET_CH, NET_CH>(d3, a2, wpart, grad + NET_OFF_W3, grad + NET_OFF_B3, n, H, Wd, s);
  hipLaunchKernelGGL((k_conv_bwd_data<NET_CH, NET_CH>), dim3(g), dim3(WG), 0, s, d3, th + NET_OFF_W3, a2, d2, n, H,
                     Wd);
  // layer 2
  wgrad<NET_CH, NET_CH>(d2, a1, wpart, grad + NET_OFF_W2, grad + NET_OFF_B2, n, H, Wd, s);
  hipLaunchKernelGGL((k_conv_bwd_data<NET_CH, NET_CH>), dim3(g), dim3(WG), 0, s, d2, th + NET_OFF_W2, a1, d1, n, H,
                     Wd);
  // layer 1 (its input is the spin map: no further backward)
  wgrad<NET_CH, 1>(d1, x, wpart, grad + NET_OFF_W1, grad + NET_OFF_B1, n, H, Wd, s);
}

void net_adam(float* th, const float* g, float* m, float* v, float lr, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(NET_NPARAM)), dim3(WG), 0, s, th, g, m, v, NET_NPARAM, lr, 0.9f, 0.999f,
                     1e-8f, t);
}

void net_gather(const int8_t* spins, const double* ratios, const int32_t* idx, int nb, int H, int Wd, int8_t* sb,
                double* rb, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_batch, dim3(nb), dim3(WG), 0, s, spins, ratios, idx, nb, H * Wd, (H - 1) * (Wd - 1),
                     sb, rb);
}

void net_cast_f64(const float* src, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_params<double>, dim3(grid_for(NET_NPARAM)), dim3(WG), 0, s, src, dst, NET_NPARAM);
}

void net_pack_bf16(const float* src, void* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_bf16, dim3(grid_for(NBF_N)), dim3(WG), 0, s, src, (char*)dst);
}

void net_local_logits(int kind, const float* w32, const double* w64, const void* wbf, const int8_t* spins, int n,
                      int H, int Wd, int flip, double* out, hipStream_t s) {
  if (kind == 2)
    hipLaunchKernelGGL((k_net_local<float, true>), dim3(n), dim3(WG), 0, s, w32, (const char*)wbf, spins, H, Wd,
                       flip, out);
  else if (kind == 1)
    hipLaunchKernelGGL((k_net_local<double, false>), dim3(n), dim3(WG), 0, s, w64, (const char*)wbf, spins, H,
                       Wd, flip, out);
  else
    hipLaunchKernelGGL((k_net_local<float, false>), dim3(n), dim3(WG), 0, s, w32, (const char*)wbf, spins, H, Wd,
                       flip, out);
}

}  // namespace vp
