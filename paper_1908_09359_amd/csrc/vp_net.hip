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

// out[b][co][y][x] = b[co] + sum W[co][ci][ky][kx] in[b][ci][y+ky-1][x+kx-1] (zero outside), ReLU if relu.
__global__ void k_conv_fwd(const float* __restrict__ in, int Ci, const float* __restrict__ W,
                           const float* __restrict__ bias, int Co, float* __restrict__ out, int n, int H, int Wd,
                           int relu) {
  const int64_t total = (int64_t)n * Co * H * Wd;
  for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < total; i += (int64_t)gridDim.x * WG) {
    const int x = (int)(i % Wd), y = (int)((i / Wd) % H);
    const int co = (int)((i / ((int64_t)H * Wd)) % Co);
    const int64_t b = i / ((int64_t)Co * H * Wd);
    float acc = bias[co];
    const float* w = W + (int64_t)co * Ci * 9;
    const float* src = in + b * Ci * H * Wd;
    for (int ci = 0; ci < Ci; ++ci) {
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const int yy = y + ky - 1;
        if (yy < 0 || yy >= H) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int xx = x + kx - 1;
          if (xx < 0 || xx >= Wd) continue;
          acc += w[ci * 9 + ky * 3 + kx] * src[((int64_t)ci * H + yy) * Wd + xx];
        }
      }
    }
    out[i] = relu ? fmaxf(acc, 0.0f) : acc;
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

// din[b][ci][y][x] = [act(b,ci,y,x) > 0] sum_{co,ky,kx} W[co][ci][ky][kx] dout[b][co][y-ky+1][x-kx+1]
__global__ void k_conv_bwd_data(const float* __restrict__ dout, int Co, const float* __restrict__ W, int Ci,
                                const float* __restrict__ act, float* __restrict__ din, int n, int H, int Wd) {
  const int64_t total = (int64_t)n * Ci * H * Wd;
  for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < total; i += (int64_t)gridDim.x * WG) {
    if (!(act[i] > 0.0f)) {
      din[i] = 0.0f;
      continue;
    }
    const int x = (int)(i % Wd), y = (int)((i / Wd) % H);
    const int ci = (int)((i / ((int64_t)H * Wd)) % Ci);
    const int64_t b = i / ((int64_t)Ci * H * Wd);
    const float* g = dout + b * Co * H * Wd;
    float acc = 0.0f;
    for (int co = 0; co < Co; ++co) {
      const float* w = W + ((int64_t)co * Ci + ci) * 9;
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const int yy = y - ky + 1;
        if (yy < 0 || yy >= H) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int xx = x - kx + 1;
          if (xx < 0 || xx >= Wd) continue;
          acc += w[ky * 3 + kx] * g[((int64_t)co * H + yy) * Wd + xx];
        }
      }
    }
    din[i] = acc;
  }
}

// One work-group per weight (co, ci, ky, kx) and per bias co:
//   gW = sum_{b,y,x} dout[b][co][y][x] in[b][ci][y+ky-1][x+kx-1],  gb = sum dout[b][co][y][x].
__global__ void k_conv_bwd_weight(const float* __restrict__ dout, int Co, const float* __restrict__ in, int Ci,
                                  float* __restrict__ gW, float* __restrict__ gb, int n, int H, int Wd) {
  const int nw = Co * Ci * 9;
  const int j = blockIdx.x;
  const int64_t HW = (int64_t)H * Wd, total = (int64_t)n * HW;
  double acc = 0.0;
  if (j < nw) {
    const int co = j / (Ci * 9), ci = (j / 9) % Ci, ky = (j % 9) / 3, kx = j % 3;
    for (int64_t i = threadIdx.x; i < total; i += WG) {
      const int64_t b = i / HW;
      const int p = (int)(i % HW), y = p / Wd + ky - 1, x = p % Wd + kx - 1;
      if (y < 0 || y >= H || x < 0 || x >= Wd) continue;
      acc += (double)dout[(b * Co + co) * HW + p] * (double)in[(b * Ci + ci) * HW + (int64_t)y * Wd + x];
    }
  } else {
    const int co = j - nw;
    for (int64_t i = threadIdx.x; i < total; i += WG) acc += (double)dout[((i / HW) * Co + co) * HW + i % HW];
  }
  acc = wg_sum(acc);
  if (threadIdx.x == 0) {
    if (j < nw) gW[j] = (float)acc;
    else gb[j - nw] = (float)acc;
  }
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

size_t net_work_floats(int n, int H, int Wd) {
  const size_t HW = (size_t)H * Wd;
  // x, a1, a2, a3, z, d3, d2, d1 (dz shares z's shape)
  return (size_t)n * HW * (1 + 3 * NET_CH + 1 + 1 + 3 * NET_CH);
}

void net_forward(const float* th, const int8_t* spins, int n, int H, int Wd, float* work, float* logits,
                 hipStream_t s) {
  const int64_t HW = (int64_t)H * Wd;
  float* x = work;
  float* a1 = x + n * HW;
  float* a2 = a1 + n * NET_CH * HW;
  float* a3 = a2 + n * NET_CH * HW;
  hipLaunchKernelGGL(k_net_input, dim3(grid_for(n * HW)), dim3(WG), 0, s, spins, n * HW, x);
  hipLaunchKernelGGL(k_conv_fwd, dim3(grid_for(n * NET_CH * HW)), dim3(WG), 0, s, x, 1, th + NET_OFF_W1,
                     th + NET_OFF_B1, NET_CH, a1, n, H, Wd, 1);
  hipLaunchKernelGGL(k_conv_fwd, dim3(grid_for(n * NET_CH * HW)), dim3(WG), 0, s, a1, NET_CH, th + NET_OFF_W2,
                     th + NET_OFF_B2, NET_CH, a2, n, H, Wd, 1);
  hipLaunchKernelGGL(k_conv_fwd, dim3(grid_for(n * NET_CH * HW)), dim3(WG), 0, s, a2, NET_CH, th + NET_OFF_W3,
                     th + NET_OFF_B3, NET_CH, a3, n, H, Wd, 1);
  hipLaunchKernelGGL(k_conv_fwd, dim3(grid_for(n * HW)), dim3(WG), 0, s, a3, NET_CH, th + NET_OFF_W4,
                     th + NET_OFF_B4, 1, logits, n, H, Wd, 0);
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
  // layer 4
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3(NET_CH * 9 + 1), dim3(WG), 0, s, dz, 1, a3, NET_CH,
                     grad + NET_OFF_W4, grad + NET_OFF_B4, n, H, Wd);
  hipLaunchKernelGGL(k_conv_bwd_data, dim3(grid_for(n * NET_CH * HW)), dim3(WG), 0, s, dz, 1, th + NET_OFF_W4,
                     NET_CH, a3, d3, n, H, Wd);
  // layer 3
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3(NET_CH * NET_CH * 9 + NET_CH), dim3(WG), 0, s, d3, NET_CH, a2, NET_CH,
                     grad + NET_OFF_W3, grad + NET_OFF_B3, n, H, Wd);
  hipLaunchKernelGGL(k_conv_bwd_data, dim3(grid_for(n * NET_CH * HW)), dim3(WG), 0, s, d3, NET_CH,
                     th + NET_OFF_W3, NET_CH, a2, d2, n, H, Wd);
  // layer 2
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3(NET_CH * NET_CH * 9 + NET_CH), dim3(WG), 0, s, d2, NET_CH, a1, NET_CH,
                     grad + NET_OFF_W2, grad + NET_OFF_B2, n, H, Wd);
  hipLaunchKernelGGL(k_conv_bwd_data, dim3(grid_for(n * NET_CH * HW)), dim3(WG), 0, s, d2, NET_CH,
                     th + NET_OFF_W2, NET_CH, a1, d1, n, H, Wd);
  // layer 1 (its input is the spin map: no further backward)
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3(NET_CH * 9 + NET_CH), dim3(WG), 0, s, d1, NET_CH, x, 1,
                     grad + NET_OFF_W1, grad + NET_OFF_B1, n, H, Wd);
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
