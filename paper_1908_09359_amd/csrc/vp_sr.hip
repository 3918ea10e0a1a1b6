// Stochastic reconfiguration step in float64 on the device.
//
//   Obar = O - <O>          (full-layout log-derivatives, samples x Np)
//   S    = Obar^T Obar / Ns + shift I
//   g    = Obar^T Ebar / Ns (= <O E> - <O><E>, Eq. (5))
//   S delta = g             (blocked right-looking Cholesky, 64x64 blocks)
//   T   <- T - lr delta
//
// The covariance and the trailing updates of the factorisation are tiled
// work-group GEMMs on f64 MFMA; only lower-triangle tiles are formed.
#include "vp_device.hpp"
#include "vp_kernels.hpp"

namespace vp {

namespace {

constexpr int NB = 64;

__device__ inline int site_of(const int64_t* coff, int N, int64_t q) {
  int lo = 0, hi = N - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (coff[mid] <= q) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ void k_sr_means(const int64_t* offs, const int64_t* coff, const int32_t* sz, int N, const T* dl,
                           const int8_t* spins, int64_t ns, int64_t nh, double* mean) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nh) return;
  const int k = site_of(coff, N, q);
  const int64_t local = q - coff[k];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = 0; i < ns; ++i) {
    double g = (double)dl[i * nh + q];
    if (spins[i * N + k]) s1 += g; else s0 += g;
  }
  mean[offs[k] + local] = s0 / (double)ns;
  mean[offs[k] + sz[k] + local] = s1 / (double)ns;
}

template <typename T>
__global__ void k_sr_center(const int64_t* offs, const int64_t* coff, const int32_t* sz, int N, const T* dl,
                            const int8_t* spins, int64_t ns, int64_t nh, int64_t np, const double* mean,
                            double* Ob) {
  const int64_t total = ns * nh;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nh, q = e - i * nh;
    const int k = site_of(coff, N, q);
    const int64_t local = q - coff[k];
    const double g = (double)dl[e];
    const int s = spins[i * N + k];
    const int64_t p0 = offs[k] + local, p1 = p0 + sz[k];
    Ob[i * np + p0] = (s == 0 ? g : 0.0) - mean[p0];
    Ob[i * np + p1] = (s == 1 ? g : 0.0) - mean[p1];
  }
}

// lower-triangle tile index t -> (bi, bj), bi >= bj
__device__ inline void tri_tile(int64_t t, int* bi, int* bj) {
  int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  *bi = (int)i;
  *bj = (int)(t - i * (i + 1) / 2);
}

// S = Obar^T Obar / ns + shift I on lower-triangle tiles
__global__ void __launch_bounds__(WG) k_sr_syrk(const double* Ob, int64_t np, int64_t ns, double* S, double shift) {
  int bi, bj;
  tri_tile(blockIdx.x, &bi, &bj);
  const int M = (int)min<int64_t>(NB, np - (int64_t)bi * NB), Nn = (int)min<int64_t>(NB, np - (int64_t)bj * NB);
  double* C = S + (int64_t)bi * NB * np + (int64_t)bj * NB;
  wg_gemm<double>(C, rowmajor((int)np), Ob + (int64_t)bi * NB, colmajor((int)np), Ob + (int64_t)bj * NB,
                  rowmajor((int)np), M, Nn, (int)ns, 1.0 / (double)ns);
  if (bi == bj)
    for (int d = threadIdx.x; d < M; d += WG) C[(int64_t)d * np + d] += shift;
}

// Cholesky of the diagonal block kb (lower), in LDS
__global__ void __launch_bounds__(WG) k_potrf_diag(double* S, int64_t np, int kb, int* flag) {
  __shared__ double a[NB][NB + 1];
  const int n = (int)min<int64_t>(NB, np - (int64_t)kb * NB);
  double* B = S + (int64_t)kb * NB * np + (int64_t)kb * NB;
  for (int e = threadIdx.x; e < n * n; e += WG) a[e / n][e % n] = B[(int64_t)(e / n) * np + e % n];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = a[j][j];
      if (!(d > 0.0) || !isfinite(d)) { *flag = 1; d = 1.0; }
      a[j][j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < n; i += WG) a[i][j] /= a[j][j];
    __syncthreads();
    const int m = n - j - 1;
    for (int e = threadIdx.x; e < m * m; e += WG) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) a[i][k] -= a[i][j] * a[k][j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * n; e += WG) {
    const int i = e / n, k = e % n;
    if (k <= i) B[(int64_t)i * np + k] = a[i][k];
  }
}

// X <- X L^{-T} for every row block below kb (one work-group per block)
__global__ void __launch_bounds__(WG) k_trsm_panel(double* S, int64_t np, int kb) {
  __shared__ double Lb[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int ib = kb + 1 + blockIdx.x;
  const int n = (int)min<int64_t>(NB, np - (int64_t)kb * NB);
  const int rows = (int)min<int64_t>(NB, np - (int64_t)ib * NB);
  const double* Lg = S + (int64_t)kb * NB * np + (int64_t)kb * NB;
  double* Xg = S + (int64_t)ib * NB * np + (int64_t)kb * NB;
  for (int e = threadIdx.x; e < n * n; e += WG) Lb[e / n][e % n] = Lg[(int64_t)(e / n) * np + e % n];
  for (int e = threadIdx.x; e < rows * n; e += WG) X[e / n][e % n] = Xg[(int64_t)(e / n) * np + e % n];
  __syncthreads();
  const int r = threadIdx.x;
  if (r < rows) {
    for (int j = 0; j < n; ++j) {
      double x = X[r][j];
      for (int m = 0; m < j; ++m) x -= X[r][m] * Lb[j][m];
      X[r][j] = x / Lb[j][j];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * n; e += WG) Xg[(int64_t)(e / n) * np + e % n] = X[e / n][e % n];
}

// A[ib][jb] -= A[ib][kb] A[jb][kb]^T for ib >= jb > kb
__global__ void __launch_bounds__(WG) k_syrk_trailing(double* S, int64_t np, int kb) {
  int ti, tj;
  tri_tile(blockIdx.x, &ti, &tj);
  const int ib = kb + 1 + ti, jb = kb + 1 + tj;
  const int M = (int)min<int64_t>(NB, np - (int64_t)ib * NB), Nn = (int)min<int64_t>(NB, np - (int64_t)jb * NB);
  const int K = (int)min<int64_t>(NB, np - (int64_t)kb * NB);
  double* C = S + (int64_t)ib * NB * np + (int64_t)jb * NB;
  const double* A = S + (int64_t)ib * NB * np + (int64_t)kb * NB;
  const double* Bt = S + (int64_t)jb * NB * np + (int64_t)kb * NB;
  wg_gemm<double>(C, rowmajor((int)np), A, rowmajor((int)np), Bt, colmajor((int)np), M, Nn, K, -1.0, true);
}

// forward solve of the diagonal block: L_kb y = b_kb (b overwritten by y)
__global__ void __launch_bounds__(WG) k_trsv_diag(const double* S, int64_t np, int kb, double* b, int backward) {
  __shared__ double Lb[NB][NB + 1];
  __shared__ double y[NB];
  const int n = (int)min<int64_t>(NB, np - (int64_t)kb * NB);
  const double* Lg = S + (int64_t)kb * NB * np + (int64_t)kb * NB;
  for (int e = threadIdx.x; e < n * n; e += WG) Lb[e / n][e % n] = Lg[(int64_t)(e / n) * np + e % n];
  for (int i = threadIdx.x; i < n; i += WG) y[i] = b[(int64_t)kb * NB + i];
  __syncthreads();
  if (!backward) {
    for (int j = 0; j < n; ++j) {
      if (threadIdx.x == 0) y[j] /= Lb[j][j];
      __syncthreads();
      for (int i = j + 1 + threadIdx.x; i < n; i += WG) y[i] -= Lb[i][j] * y[j];
      __syncthreads();
    }
  } else {  // L_kb^T x = b
    for (int j = n - 1; j >= 0; --j) {
      if (threadIdx.x == 0) y[j] /= Lb[j][j];
      __syncthreads();
      for (int i = threadIdx.x; i < j; i += WG) y[i] -= Lb[j][i] * y[j];
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += WG) b[(int64_t)kb * NB + i] = y[i];
}

// forward: b_i -= sum_m L[i][kb*NB+m] y_m for rows below block kb
// backward: b_i -= sum_m L[kb*NB+m][i] x_m for rows above block kb
__global__ void k_gemv_update(const double* S, int64_t np, int kb, double* b, int backward) {
  const int n = (int)min<int64_t>(NB, np - (int64_t)kb * NB);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c0 = (int64_t)kb * NB;
  if (!backward) {
    const int64_t row = c0 + NB + i;
    if (row >= np) return;
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc += S[row * np + c0 + m] * b[c0 + m];
    b[row] -= acc;
  } else {
    if (i >= c0) return;
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc += S[(c0 + m) * np + i] * b[c0 + m];
    b[i] -= acc;
  }
}

__global__ void k_sr_apply(double* T, const double* delta, int64_t np, double lr, double* delta_out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    T[p] -= lr * delta[p];
    if (delta_out) delta_out[p] = delta[p];
  }
}

}  // namespace

template <typename T>
int launch_sr(const int64_t* offs, const int64_t* coff, const int32_t* sz, int N, int64_t np, const double* e,
              const T* dl, const int8_t* spins, int64_t ns, double shift, double lr, double* Tm,
              double* delta_out, double* work, int* flag, hipStream_t s) {
  // work layout: mean [np] | g [np] | emean [1] | Obar [ns*np] | S [np*np]
  const int64_t nh = np / 2;
  double* mean = work;
  double* g = mean + np;
  double* emean = g + np;
  double* Ob = emean + 8;
  double* Sm = Ob + ns * np;
  const int nt = (int)((np + NB - 1) / NB);
  hipLaunchKernelGGL(k_sr_means<T>, dim3((unsigned)((nh + WG - 1) / WG)), dim3(WG), 0, s, offs, coff, sz, N, dl,
                     spins, ns, nh, mean);
  hipLaunchKernelGGL(k_sr_center<T>, dim3(8192), dim3(WG), 0, s, offs, coff, sz, N, dl, spins, ns, nh, np, mean, Ob);
  launch_gradient<T>(offs, coff, sz, N, np, e, dl, spins, ns, g, emean, nullptr, s);
  hipLaunchKernelGGL(k_sr_syrk, dim3((unsigned)((int64_t)nt * (nt + 1) / 2)), dim3(WG), 0, s, (const double*)Ob, np,
                     ns, Sm, shift);
  for (int kb = 0; kb < nt; ++kb) {
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(WG), 0, s, Sm, np, kb, flag);
    const int rest = nt - kb - 1;
    if (rest > 0) {
      hipLaunchKernelGGL(k_trsm_panel, dim3(rest), dim3(WG), 0, s, Sm, np, kb);
      hipLaunchKernelGGL(k_syrk_trailing, dim3((unsigned)((int64_t)rest * (rest + 1) / 2)), dim3(WG), 0, s, Sm, np,
                         kb);
    }
  }
  for (int kb = 0; kb < nt; ++kb) {
    hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(WG), 0, s, (const double*)Sm, np, kb, g, 0);
    const int64_t rows = np - (int64_t)(kb + 1) * NB;
    if (rows > 0)
      hipLaunchKernelGGL(k_gemv_update, dim3((unsigned)((rows + WG - 1) / WG)), dim3(WG), 0, s, (const double*)Sm, np,
                         kb, g, 0);
  }
  for (int kb = nt - 1; kb >= 0; --kb) {
    hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(WG), 0, s, (const double*)Sm, np, kb, g, 1);
    const int64_t rows = (int64_t)kb * NB;
    if (rows > 0)
      hipLaunchKernelGGL(k_gemv_update, dim3((unsigned)((rows + WG - 1) / WG)), dim3(WG), 0, s, (const double*)Sm, np,
                         kb, g, 1);
  }
  hipLaunchKernelGGL(k_sr_apply, dim3((unsigned)std::min<int64_t>((np + WG - 1) / WG, 65536)), dim3(WG), 0, s, Tm,
                     (const double*)g, np, lr, delta_out);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

int64_t sr_work_doubles(int64_t np, int64_t ns) { return 2 * np + 8 + ns * np + np * np; }

template int launch_sr<double>(const int64_t*, const int64_t*, const int32_t*, int, int64_t, const double*,
                               const double*, const int8_t*, int64_t, double, double, double*, double*, double*,
                               int*, hipStream_t);
template int launch_sr<float>(const int64_t*, const int64_t*, const int32_t*, int, int64_t, const double*,
                              const float*, const int8_t*, int64_t, double, double, double*, double*, double*, int*,
                              hipStream_t);

}  // namespace vp
