// Building blocks of the variational boundary fit (App. B: the boundary MPS
// that minimises ||M |U> - |U'>||^2, found by sweeps of single-site updates):
// its start, the thin Householder QR that keeps the fitted sites orthonormal,
// and the move of the LQ factor of the start into the neighbouring site.
//
// A fitted site is stored like every boundary site, padded [c][d][c]; its true
// extent is k_left x p x k_right.  The QR and LQ act on that compact block,
// addressed through a strided view (element (i, j) at site[vaddr(v, i, j)]).
#pragma once

#include "vp_device.hpp"
#include "vp_eig.hpp"

namespace vp {

// Start of the fit: the leading kl x kr block of the product site
// B[(a,l)][y][(b,r)] = sum_x A[a][x][b] t[l][x][r][y] (combined indices
// a Dl + l and b Dr + r, Dl / Dr the true dims of the row's l / r legs),
// zero outside k < kl, k' < kr, y < P.  out: padded c x d x c.
template <typename T>
__device__ void fit_start(T* __restrict__ out_p, const T* __restrict__ A_p, S3 sA, const T* __restrict__ t_p, S4 st,
                          int c, int d, int kl, int kr, int P, int Dl, int Dr) {
  auto* out = gmem(out_p);
  const auto* A = gmem(A_p);
  const auto* t = gmem(t_p);
  const int n = c * d * c;
  for (int e = threadIdx.x; e < n; e += WG) {
    const int k = e / (d * c), y = (e / c) % d, k2 = e % c;
    double v = 0.0;
    if (k < kl && k2 < kr && y < P) {
      const int a = k / Dl, l = k % Dl, b = k2 / Dr, r = k2 % Dr;
      for (int x = 0; x < d; ++x)
        v += (double)A[a * sA.s0 + x * sA.s1 + b * sA.s2] * (double)t[l * st.l + x * st.u + r * st.r + y * st.d];
    }
    out[e] = (T)v;
  }
  __syncthreads();
}

// Thin Householder QR (the reflectors of Golub & Van Loan, Sec. 5.2) of the
// m x n matrix (m >= n) whose entry (i, j) lies at site[vaddr(v, i, j)]:
// the site (site_elems entries, zero outside the view) is overwritten by Q,
// m x n with orthonormal columns, through the same view.  X and Q are global
// scratch of m n elements each (column-major, ld m); on return the upper
// triangle of X holds R.  Reductions in float64, fixed order.
template <typename T>
__device__ void fit_qr(T* __restrict__ site_p, int site_elems, View v, int m, int n, T* __restrict__ X_p,
                       T* __restrict__ Q_p) {
  auto* site = gmem(site_p);
  auto* X = gmem(X_p);
  auto* Q = gmem(Q_p);
  __shared__ double tau_s[64];
  __shared__ double w_s[64];
  const int tid = threadIdx.x;
  for (int e = tid; e < m * n; e += WG) X[e] = site[vaddr(v, e % m, e / m)];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = j + 1 + tid; i < m; i += WG) s += (double)X[i + j * m] * (double)X[i + j * m];
    s = wg_sum(s);
    const double alpha = X[j + j * m];
    double beta = alpha, tau = 0.0, scal = 0.0;
    if (s > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + s), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    __syncthreads();  // every thread has read alpha
    for (int i = j + 1 + tid; i < m; i += WG) X[i + j * m] = (T)((double)X[i + j * m] * scal);
    if (tid == 0) {
      X[j + j * m] = (T)beta;
      tau_s[j] = tau;
    }
    __syncthreads();
    if (tau != 0.0 && j + 1 < n) {
      // w_k = tau (x_jk + sum_{i>j} v_i x_ik), 16 lanes per column
      for (int k0 = j + 1; k0 < n; k0 += WG / 16) {
        const int k = k0 + (tid >> 4);
        double p = 0.0;
        if (k < n)
          for (int i = j + 1 + (tid & 15); i < m; i += 16) p += (double)X[i + j * m] * (double)X[i + k * m];
        p = row16_sum(p);
        if ((tid & 15) == 0 && k < n) w_s[k] = tau * ((double)X[j + k * m] + p);
      }
      __syncthreads();
      const int rows = m - j;
      for (int e = tid; e < rows * (n - j - 1); e += WG) {
        const int i = j + e % rows, k = j + 1 + e / rows;
        const double vi = i == j ? 1.0 : (double)X[i + j * m];
        X[i + k * m] = (T)((double)X[i + k * m] - vi * w_s[k]);
      }
      __syncthreads();
    }
  }
  // Q = H_0 H_1 ... H_{n-1} applied to the first n columns of the identity
  for (int e = tid; e < m * n; e += WG) Q[e] = (T)((e % m) == (e / m) ? 1.0 : 0.0);
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    if (tau == 0.0) continue;  // uniform
    for (int k0 = j; k0 < n; k0 += WG / 16) {
      const int k = k0 + (tid >> 4);
      double p = 0.0;
      if (k < n)
        for (int i = j + (tid & 15); i < m; i += 16) p += (i == j ? 1.0 : (double)X[i + j * m]) * (double)Q[i + k * m];
      p = row16_sum(p);
      if ((tid & 15) == 0 && k < n) w_s[k] = tau * p;
    }
    __syncthreads();
    const int rows = m - j;
    for (int e = tid; e < rows * (n - j); e += WG) {
      const int i = j + e % rows, k = j + e / rows;
      const double vi = i == j ? 1.0 : (double)X[i + j * m];
      Q[i + k * m] = (T)((double)Q[i + k * m] - vi * w_s[k]);
    }
    __syncthreads();
  }
  for (int e = tid; e < site_elems; e += WG) site[e] = T(0);
  __syncthreads();
  for (int e = tid; e < m * n; e += WG) site[vaddr(v, e % m, e / m)] = Q[e];
  __syncthreads();
}

// The LQ factor L = R^T of the site just made right-orthonormal (R from the
// QR of its transpose, the upper triangle of X, ld m, n x n) moved into its
// left neighbour: nb[(k, p)][q] <- sum_{r >= q} nb[(k, p)][r] R[q][r] for
// k < kl, p < P, q < n.  tmp: global scratch of c d c elements.
template <typename T>
__device__ void fit_carry(T* __restrict__ nb_p, const T* __restrict__ X_p, int m, int n, int kl, int P, int c, int d,
                          T* __restrict__ tmp_p) {
  auto* nb = gmem(nb_p);
  const auto* X = gmem(X_p);
  auto* tmp = gmem(tmp_p);
  const int tid = threadIdx.x;
  for (int e = tid; e < kl * P * n; e += WG) {
    const int q = e % n, kp = e / n, k = kp / P, p = kp % P;
    const int base = k * (d * c) + p * c;
    double s = 0.0;
    for (int r = q; r < n; ++r) s += (double)nb[base + r] * (double)X[q + r * m];
    tmp[e] = (T)s;
  }
  __syncthreads();
  for (int e = tid; e < kl * P * n; e += WG) {
    const int q = e % n, kp = e / n, k = kp / P, p = kp % P;
    nb[k * (d * c) + p * c + q] = tmp[e];
  }
  __syncthreads();
}

}  // namespace vp

namespace vp {

// Sum over the 64 lanes of a wavefront, returned to every lane.
__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

constexpr int FIT_WAVE_N = 16;  // columns the one-wavefront QR holds in registers

// fit_qr for m <= 128 and n <= FIT_WAVE_N, by the first wavefront alone: lane
// l holds rows l and l + 64 of every column in registers, each reflector's
// norms and column sums are wavefront reductions (no barrier, no LDS).  Same
// reflectors, same Q (through the view) and R (the upper triangle of X,
// column-major, ld m) as fit_qr.  All threads of the work-group call it.
template <typename T>
__device__ void fit_qr_wave(T* __restrict__ site_p, int site_elems, View v, int m, int n, T* __restrict__ X_p) {
  auto* site = gmem(site_p);
  auto* X = gmem(X_p);
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int lane = tid;
    double x[2][FIT_WAVE_N], q[2][FIT_WAVE_N], tau[FIT_WAVE_N];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < FIT_WAVE_N; ++k) {
        const int i = lane + 64 * h;
        x[h][k] = (i < m && k < n) ? (double)site[vaddr(v, i, k)] : 0.0;
      }
#pragma unroll
    for (int j = 0; j < FIT_WAVE_N; ++j) {
      tau[j] = 0.0;
      if (j < n) {
        double s = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = lane + 64 * h;
          s += (i > j && i < m) ? x[h][j] * x[h][j] : 0.0;
        }
        s = wave_sum(s);
        const double alpha = __shfl(x[0][j], j, 64);  // row j < 16 sits in lane j, slot 0
        double beta = alpha, t = 0.0, scal = 0.0;
        if (s > 0.0) {
          beta = -copysign(sqrt(alpha * alpha + s), alpha);
          t = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        tau[j] = t;
        // v: 1 at row j, x scal below it, 0 above; stored in column j below the diagonal, beta on it
        double vv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = lane + 64 * h;
          vv[h] = i == j ? 1.0 : ((i > j && i < m) ? x[h][j] * scal : 0.0);
          x[h][j] = i == j ? beta : (i > j ? vv[h] : x[h][j]);
        }
        if (t != 0.0) {
          double w[FIT_WAVE_N];
#pragma unroll
          for (int k = 0; k < FIT_WAVE_N; ++k) w[k] = (k > j) ? vv[0] * x[0][k] + vv[1] * x[1][k] : 0.0;
#pragma unroll
          for (int k = 0; k < FIT_WAVE_N; ++k)
            if (k > j) w[k] = t * wave_sum(w[k]);
#pragma unroll
          for (int k = 0; k < FIT_WAVE_N; ++k)
            if (k > j) {
              x[0][k] -= vv[0] * w[k];
              x[1][k] -= vv[1] * w[k];
            }
        }
      }
    }
    // Q = H_0 ... H_{n-1} [I; 0]
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < FIT_WAVE_N; ++k) q[h][k] = (lane + 64 * h == k) ? 1.0 : 0.0;
#pragma unroll
    for (int j = FIT_WAVE_N - 1; j >= 0; --j) {
      if (j < n && tau[j] != 0.0) {
        double vv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = lane + 64 * h;
          vv[h] = i == j ? 1.0 : ((i > j && i < m) ? x[h][j] : 0.0);
        }
        double w[FIT_WAVE_N];
#pragma unroll
        for (int k = 0; k < FIT_WAVE_N; ++k) w[k] = (k >= j && k < n) ? vv[0] * q[0][k] + vv[1] * q[1][k] : 0.0;
#pragma unroll
        for (int k = 0; k < FIT_WAVE_N; ++k)
          if (k >= j && k < n) w[k] = tau[j] * wave_sum(w[k]);
#pragma unroll
        for (int k = 0; k < FIT_WAVE_N; ++k)
          if (k >= j && k < n) {
            q[0][k] -= vv[0] * w[k];
            q[1][k] -= vv[1] * w[k];
          }
      }
    }
    // R (upper triangle) for the carry
#pragma unroll
    for (int k = 0; k < FIT_WAVE_N; ++k)
      if (k < n && lane <= k) X[lane + k * m] = (T)x[0][k];
    for (int e = lane; e < site_elems; e += 64) site[e] = T(0);
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < FIT_WAVE_N; ++k) {
        const int i = lane + 64 * h;
        if (i < m && k < n) site[vaddr(v, i, k)] = (T)q[h][k];
      }
  }
  __syncthreads();
}

// The thin QR of the fit: one wavefront when the block fits its registers.
template <typename T>
__device__ inline void fit_qr_any(T* site, int site_elems, View v, int m, int n, T* X, T* Q) {
  if (m <= 128 && n <= FIT_WAVE_N) fit_qr_wave<T>(site, site_elems, v, m, n, X);
  else fit_qr<T>(site, site_elems, v, m, n, X, Q);
}

}  // namespace vp
