// Leading eigenpairs of a small symmetric matrix, one work-group per matrix.
//
// Householder tridiagonalisation (the unblocked symmetric reduction of Golub &
// Van Loan, Sec. 8.3.1) on the packed lower triangle held in LDS, eigenvalues
// of the tridiagonal matrix by Sturm-count multisection (16 probes per
// eigenvalue and step), eigenvectors of the tridiagonal matrix by inverse
// iteration with partial-pivoting LU (Wilkinson), modified Gram-Schmidt among
// the kept vectors, and back-transformation by the stored reflectors.
#pragma once
#include "vp_device.hpp"

namespace vp {

constexpr int EIG_NMAX = 128;
constexpr int EIG_KMAX = 16;   // eigenvectors per inverse-iteration batch (one thread each)
constexpr int EIG_PACK = EIG_NMAX * (EIG_NMAX + 1) / 2;
// LDS the caller provides: the packed matrix; afterwards the same space holds
// the LU factors (3 x n x EIG_KMAX), the kept vectors (n x EIG_KMAX) and the
// pivot-swap bit words (n).
// Small work arrays follow the packed matrix: d, e, e^2, tau, p, w, v (7 n),
// two half-row partials (2 n), the multisection probes and counts (2 WG) and
// the batch eigenvalues (EIG_KMAX).
constexpr size_t EIG_PACK_BYTES = sizeof(double) * EIG_PACK;
constexpr size_t EIG_SMALL_BYTES = sizeof(double) * (9 * EIG_NMAX + WG + EIG_KMAX) + sizeof(int) * WG;
constexpr size_t EIG_LDS_BYTES = EIG_PACK_BYTES + EIG_SMALL_BYTES;
static_assert(3 * EIG_NMAX * EIG_KMAX * 8 + EIG_NMAX * EIG_KMAX * 8 + EIG_NMAX * 4 <= EIG_PACK_BYTES, "eig LDS");

__device__ inline int tri(int i) { return i * (i + 1) / 2; }

// Number of eigenvalues of tridiag(d, e) strictly below x (Sturm sequence).
__device__ inline int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int j = 1; j < n; ++j) {
    q = d[j] - x - e2[j - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// H: n x n symmetric, row-major (ld n), any address space; n <= EIG_NMAX.
// Writes the eigenvectors of the k largest eigenvalues, in descending order,
// as columns 0..k-1 of V (ld k) and the eigenvalues to lam[0..k-1].
// refl: global scratch of at least EIG_PACK doubles (Householder vectors);
// lds: EIG_LDS_BYTES of LDS owned by the caller.
__device__ void sym_topk_eig(const double* H, int n, int k, double* V, double* lam, double* refl, char* lds) {
  double* Ap = reinterpret_cast<double*>(lds);
  double* Xs = Ap + 3 * EIG_NMAX * EIG_KMAX;                            // after the tridiagonalisation
  unsigned* pivw = reinterpret_cast<unsigned*>(Xs + EIG_NMAX * EIG_KMAX);  // bit t: row swap of vector t
  double* dg = reinterpret_cast<double*>(lds + EIG_PACK_BYTES);
  double* eg = dg + EIG_NMAX;
  double* e2 = eg + EIG_NMAX;
  double* tau = e2 + EIG_NMAX;
  double* pv = tau + EIG_NMAX;
  double* wv = pv + EIG_NMAX;
  double* vv = wv + EIG_NMAX;
  double (*pv2)[EIG_NMAX] = reinterpret_cast<double (*)[EIG_NMAX]>(vv + EIG_NMAX);
  double* probe_x = vv + 3 * EIG_NMAX;
  double* lamb = probe_x + WG;
  int* probe_c = reinterpret_cast<int*>(lamb + EIG_KMAX);
  const int tid = threadIdx.x;

  for (int e = tid; e < n * n; e += WG) {
    int i = e / n, j = e - i * n;
    if (j <= i) Ap[tri(i) + j] = H[e];
  }
  __syncthreads();

  // ---- tridiagonalisation: Q^T A Q = T, Q = H_0 H_1 ... H_{n-3}
  for (int i = 0; i < n - 2; ++i) {
    const double alpha = Ap[tri(i + 1) + i];
    double xn2 = 0.0;
    for (int r = i + 2 + tid; r < n; r += WG) xn2 += Ap[tri(r) + i] * Ap[tri(r) + i];
    xn2 = wg_sum(xn2);
    double beta = alpha, t = 0.0;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      t = (beta - alpha) / beta;
      const double scal = 1.0 / (alpha - beta);
      for (int r = i + 2 + tid; r < n; r += WG) Ap[tri(r) + i] *= scal;
    }
    __syncthreads();  // the loop below reads entries scaled by other threads
    // reflector i: v[i+1] = 1, v[r] = Ap[r][i] (r > i+1); also kept in global memory
    for (int r = i + 1 + tid; r < n; r += WG) {
      double v = (r == i + 1) ? 1.0 : Ap[tri(r) + i];
      vv[r] = v;
      refl[tri(r) + i] = v;
    }
    if (tid == 0) { dg[i] = Ap[tri(i) + i]; eg[i] = beta; tau[i] = t; }
    __syncthreads();
    if (t != 0.0) {
      // p = t * A22 v over rows/cols i+1..n-1: two threads per row (interleaved columns)
      {
        const int r = i + 1 + (tid >> 1), h = tid & 1;
        double acc = 0.0;
        if (r < n) {
          const int trr = tri(r);
#pragma unroll 8
          for (int s = i + 1 + h; s < n; s += 2) acc += (s <= r ? Ap[trr + s] : Ap[tri(s) + r]) * vv[s];
          pv2[h][r] = acc;
        }
      }
      __syncthreads();
      double pw = 0.0;
      for (int r = i + 1 + tid; r < n; r += WG) {
        const double p = t * (pv2[0][r] + pv2[1][r]);
        pv[r] = p;
        pw += p * vv[r];
      }
      const double K = -0.5 * t * wg_sum(pw);
      for (int r = i + 1 + tid; r < n; r += WG) wv[r] = pv[r] + K * vv[r];
      __syncthreads();
      // A22 -= v w^T + w v^T on the lower triangle, two threads per row
      {
        const int r = i + 1 + (tid >> 1), h = tid & 1;
        if (r < n) {
          const int trr = tri(r);
          const double vr = vv[r], wr = wv[r];
#pragma unroll 8
          for (int s = i + 1 + h; s <= r; s += 2) Ap[trr + s] -= vr * wv[s] + wr * vv[s];
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (n >= 2) {
      dg[n - 2] = Ap[tri(n - 2) + n - 2];
      eg[n - 2] = Ap[tri(n - 1) + n - 2];
      tau[n - 2] = 0.0;
    }
    dg[n - 1] = Ap[tri(n - 1) + n - 1];
    eg[n - 1] = 0.0;
    tau[n - 1] = 0.0;
  }
  __syncthreads();
  for (int j = tid; j < n; j += WG) e2[j] = eg[j] * eg[j];

  // ---- Gershgorin interval and pivot floor
  double lo = 1e300, hi = -1e300, amax = 0.0;
  for (int j = tid; j < n; j += WG) {
    double r = (j > 0 ? fabs(eg[j - 1]) : 0.0) + (j < n - 1 ? fabs(eg[j]) : 0.0);
    lo = fmin(lo, dg[j] - r);
    hi = fmax(hi, dg[j] + r);
    amax = fmax(amax, fmax(fabs(dg[j]), fabs(eg[j])));
  }
  lo = -wg_max(-lo);
  hi = wg_max(hi);
  amax = wg_max(amax);
  const double span = fmax(hi - lo, 1e-300);
  lo -= 2.2e-16 * span + 1e-300;
  hi += 2.2e-16 * span + 1e-300;
  const double pivmin = fmax(1e-300, 2.2e-16 * 2.2e-16 * amax * amax);
  const double tiny = fmax(1e-300, 2.2e-16 * amax);

  for (int b0 = 0; b0 < k; b0 += EIG_KMAX) {
    const int kb = min(EIG_KMAX, k - b0);
    // ---- eigenvalues b0 .. b0+kb-1 (descending): 16 probes per eigenvalue
    const int g = tid >> 4, lane = tid & 15;
    const int t = b0 + g;
    const int q = n - 1 - t;            // ascending index
    double a = lo, c = hi;
    for (int it = 0; it < 13; ++it) {  // 17^13 > 2^52
      double x = a + (c - a) * (double)(lane + 1) / 17.0;
      int cnt = (g < kb) ? sturm_count(dg, e2, n, x, pivmin) : 0;
      probe_x[tid] = x;
      probe_c[tid] = cnt;
      __syncthreads();
      if (g < kb) {
        double na = a, nc = c;
        for (int s = 0; s < 16; ++s) {
          int cs = probe_c[(g << 4) + s];
          double xs = probe_x[(g << 4) + s];
          if (cs <= q) na = xs;
          else { nc = xs; break; }
        }
        a = na;
        c = nc;
      }
      __syncthreads();
    }
    if (g < kb && lane == 0) lamb[g] = 0.5 * (a + c);
    __syncthreads();

    // ---- inverse iteration, one thread per eigenvector; LU factors in LDS (Ap is free now)
    double* U0 = Ap;                               // reciprocal pivots
    double* U1 = Ap + 1 * EIG_NMAX * EIG_KMAX;     // first superdiagonal of U
    double* ML = Ap + 2 * EIG_NMAX * EIG_KMAX;     // multipliers
    for (int j = tid; j < n; j += WG) pivw[j] = 0u;
    __syncthreads();
    if (tid < kb) {
      const int col = b0 + tid;
      const double lm = lamb[tid];
#define IX(j) ((j) * EIG_KMAX + tid)
      // Gaussian elimination with partial pivoting of T - lm I; a swap of rows j
      // and j+1 puts the known entry e[j+1] on the second superdiagonal.
      double aa = dg[0] - lm, cc = n > 1 ? eg[0] : 0.0;
      for (int j = 0; j < n - 1; ++j) {
        const double bb = eg[j];
        const double a1 = dg[j + 1] - lm;
        const double c1 = (j + 1 < n - 1) ? eg[j + 1] : 0.0;
        if (fabs(aa) >= fabs(bb)) {
          const double piv = fabs(aa) < tiny ? (aa < 0.0 ? -tiny : tiny) : aa;
          const double m = bb / piv;
          U0[IX(j)] = 1.0 / piv; U1[IX(j)] = cc; ML[IX(j)] = m;
          aa = a1 - m * cc;
          cc = c1;
        } else {
          const double m = aa / bb;
          U0[IX(j)] = 1.0 / bb; U1[IX(j)] = a1; ML[IX(j)] = m;
          atomicOr(&pivw[j], 1u << tid);
          const double naa = cc - m * a1;
          cc = -m * c1;
          aa = naa;
        }
      }
      U0[IX(n - 1)] = 1.0 / (fabs(aa) < tiny ? (aa < 0.0 ? -tiny : tiny) : aa);
      // deterministic, eigenvector-dependent start vector
      for (int j = 0; j < n; ++j) {
        uint64_t h = (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull ^ (uint64_t)(col + 1) * 0xD2E7470EE14C6C93ull;
        h ^= h >> 29;
        Xs[IX(j)] = 0.5 + (double)(h & 0xFFFF) / 65536.0;
      }
      for (int it = 0; it < 3; ++it) {
        for (int j = 0; j < n - 1; ++j) {
          double rj = Xs[IX(j)], rj1 = Xs[IX(j + 1)];
          if ((pivw[j] >> tid) & 1u) { double tt = rj; rj = rj1; rj1 = tt; }
          Xs[IX(j)] = rj;
          Xs[IX(j + 1)] = rj1 - ML[IX(j)] * rj;
        }
        double x1 = 0.0, x2 = 0.0, nrm = 0.0;
        for (int j = n - 1; j >= 0; --j) {
          const double u2 = ((pivw[j] >> tid) & 1u) && j + 1 < n - 1 ? eg[j + 1] : 0.0;
          const double xj = (Xs[IX(j)] - U1[IX(j)] * x1 - u2 * x2) * U0[IX(j)];  // U0 holds 1/pivot
          Xs[IX(j)] = xj;
          x2 = x1;
          x1 = xj;
          nrm = fmax(nrm, fabs(xj));
        }
        const double inv = nrm > 0.0 ? 1.0 / nrm : 1.0;
        for (int j = 0; j < n; ++j) Xs[IX(j)] *= inv;
      }
#undef IX
    }
    __syncthreads();
    if (tid < kb) lam[b0 + tid] = lamb[tid];
    if (k > EIG_KMAX) {
      // more than one batch: park this batch in V (global) and finish there
      for (int e = tid; e < n * kb; e += WG) {
        int j = e / kb, tt = e - j * kb;
        V[(int64_t)j * k + b0 + tt] = Xs[j * EIG_KMAX + tt];
      }
    }
    __syncthreads();
  }

  // Vectors live in LDS (Xs, [j][t]) when k <= EIG_KMAX, else in V.
  const bool in_lds = k <= EIG_KMAX;
  const int ld = in_lds ? EIG_KMAX : k;
  double* Vw = in_lds ? Xs : V;

  // ---- classical Gram-Schmidt, twice, over the kept vectors in descending order
  for (int col = 1; col < k; ++col) {
    for (int pass = 0; pass < 2; ++pass) {
      // dots with every earlier vector: 16 lanes per earlier vector
      for (int s0 = 0; s0 < col; s0 += WG / 16) {
        const int sv = s0 + (tid >> 4);
        double dp = 0.0;
        if (sv < col)
          for (int j = tid & 15; j < n; j += 16) dp += Vw[j * ld + sv] * Vw[j * ld + col];
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) dp += __shfl_xor(dp, o, 16);
        if ((tid & 15) == 0 && sv < col) pv[sv] = dp;
      }
      __syncthreads();
      for (int j = tid; j < n; j += WG) {
        double x = Vw[j * ld + col];
        for (int sv = 0; sv < col; ++sv) x -= pv[sv] * Vw[j * ld + sv];
        Vw[j * ld + col] = x;
      }
      __syncthreads();
    }
  }
  for (int c0 = 0; c0 < k; c0 += WG / 16) {
    const int col = c0 + (tid >> 4);
    double nn = 0.0;
    if (col < k)
      for (int j = tid & 15; j < n; j += 16) nn += Vw[j * ld + col] * Vw[j * ld + col];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 16);
    if ((tid & 15) == 0 && col < k) pv[col] = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < n * k; e += WG) {
    const int j = e / k, col = e - j * k;
    Vw[j * ld + col] *= pv[col];
  }
  __syncthreads();

  // ---- back-transformation: x <- H_0 H_1 ... H_{n-3} x; reflector i streamed from global
  // memory, the next one prefetched into a register while the current one is applied
  double vreg = (n >= 3 && tid > n - 3 && tid < n) ? refl[tri(tid) + n - 3] : 0.0;
  for (int i = n - 3; i >= 0; --i) {
    if (tid < n) vv[tid] = tid > i ? vreg : 0.0;
    if (i >= 1 && tid > i - 1 && tid < n) vreg = refl[tri(tid) + i - 1];
    __syncthreads();
    const double t = tau[i];
    if (t != 0.0) {
      for (int c0 = 0; c0 < k; c0 += WG / 16) {
        const int col = c0 + (tid >> 4);
        double dp = 0.0;
        if (col < k)
          for (int r = i + 1 + (tid & 15); r < n; r += 16) dp += vv[r] * Vw[r * ld + col];
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) dp += __shfl_xor(dp, o, 16);
        if ((tid & 15) == 0 && col < k) pv[col] = t * dp;
      }
      __syncthreads();
      for (int e = tid; e < (n - i - 1) * k; e += WG) {
        const int rr = e / k, col = e - rr * k;
        const int r = i + 1 + rr;
        Vw[r * ld + col] -= pv[col] * vv[r];
      }
    }
    __syncthreads();
  }
  if (in_lds) {
    for (int e = tid; e < n * k; e += WG) {
      const int j = e / k, col = e - j * k;
      V[(int64_t)j * k + col] = Xs[j * EIG_KMAX + col];
    }
    __syncthreads();
  }
}

}  // namespace vp
