// Leading eigenpairs of a small symmetric matrix, one work-group per matrix.
//
// Householder tridiagonalisation (the unblocked symmetric reduction of Golub &
// Van Loan, Sec. 8.3.1) with the matrix in registers, eigenvalues of the
// tridiagonal matrix by Sturm-count multisection (16 probes per eigenvalue and
// step), eigenvectors of the tridiagonal matrix by inverse iteration with
// partial-pivoting LU (Wilkinson), classical Gram-Schmidt (twice, each vector
// normalised as soon as it is orthogonalised) among the kept vectors, and
// back-transformation by the stored reflectors.
//
// Global and LDS data are addressed through address-space-qualified pointers
// wherever the compiler cannot infer the space: a generic (flat) access counts
// on the LDS wait counter as well, so every later LDS wait would also wait for
// outstanding global stores.
#pragma once
#include "vp_device.hpp"

namespace vp {

constexpr int EIG_NMAX = 128;
constexpr int EIG_KMAX = 16;   // eigenvectors per inverse-iteration batch (one thread each)
constexpr int EIG_INV_ITERS = 2;  // inverse-iteration sweeps per eigenvector (shifts accurate to the last bits)
constexpr int EIG_PACK = EIG_NMAX * (EIG_NMAX + 1) / 2;
// LDS the caller provides: a first block (the size of a packed matrix) that
// holds the LU factors (3 x n x EIG_KMAX) and the kept vectors (n x EIG_KMAX).
// Small work arrays follow the packed matrix: d, e, e^2, tau, p, w, v (7 n),
// two spare rows (2 n), a row of WG doubles (reduction partials, the iterates'
// scales) and the batch eigenvalues (EIG_KMAX).
constexpr size_t EIG_PACK_BYTES = sizeof(double) * EIG_PACK;
constexpr size_t EIG_SMALL_BYTES = sizeof(double) * (9 * EIG_NMAX + WG + EIG_KMAX);
constexpr size_t EIG_LDS_BYTES = EIG_PACK_BYTES + EIG_SMALL_BYTES;
static_assert(3 * EIG_NMAX * EIG_KMAX * 8 + EIG_NMAX * EIG_KMAX * 8 <= EIG_PACK_BYTES, "eig LDS");

__device__ inline int tri(int i) { return i * (i + 1) / 2; }

// Number of eigenvalues of tridiag(d, e) strictly below x (Sturm sequence).
// 1/q: the hardware reciprocal refined by one Newton step (relative error at
// the level of the last bits; the counts and pivots below need no more).
__device__ inline double recip(double q) {
  const double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}

__device__ inline int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
#pragma unroll 8
  for (int j = 1; j < n; ++j) {
    q = d[j] - x - e2[j - 1] * recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(1))) double gbl_f64;

// x from the lane given by the DPP control `ctrl` within its row of 16 lanes.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 16 lanes of a row, returned to all of them: quad_perm [1,0,3,2]
// and [2,3,0,1] sum each quad, row_half_mirror pairs the quads of each half,
// row_mirror the halves.
__device__ inline double row16_sum(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x141>(x);
  x += dpp_f64<0x140>(x);
  return x;
}

// x + x of lane l ^ 32 and x + x of lane l ^ 16, by the gfx950 lane swaps
// (v_permlane32_swap / v_permlane16_swap on each half of the double): VALU
// moves, no LDS round trip.  With x as both operands, the swap leaves the
// lane's own value in one result and its partner's in the other.
__device__ inline double xor32_sum(double x) {
  const long long b = __double_as_longlong(x);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  return __longlong_as_double(((long long)hi[0] << 32) | lo[0]) + __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}
__device__ inline double xor16_sum(double x) {
  const long long b = __double_as_longlong(x);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  return __longlong_as_double(((long long)hi[0] << 32) | lo[0]) + __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// Householder tridiagonalisation Q^T A Q = T, Q = H_0 H_1 ... H_{n-3}.
// The full symmetric matrix lives in registers: thread t owns the 8x8 tile
// (t / 16, t % 16) of the 128 x 128 zero-padded matrix, so the 16 tiles of a
// block row sit in one row of 16 lanes of a wavefront.  Step i applies
// H_i A H_i = A - v w^T - w v^T to the whole matrix (v vanishes on rows <= i,
// which leaves the finished rows and columns as they are up to rounding).
// Per step: the owners of column i publish it with partial norms; every
// thread forms the reflector; p = t A v by tile products summed over the row
// of lanes; v^T p over the block rows through LDS; then the rank-2 update.
// H: n x n row-major (ld n); outputs d (dg), e (eg), tau and the reflectors
// refl[tri(r) + i] = v_r (r > i, v_{i+1} = 1); xc0, xc1, pv: LDS rows of
// EIG_NMAX doubles, red: 36 doubles of LDS.  Column i and its norms alternate
// between two buffers, so a step needs two barriers.  All threads of the
// work-group call it.
__device__ __noinline__ void eig_tridiag(const gbl_f64* H, int n, lds_f64* dg, lds_f64* eg, lds_f64* tau,
                                         lds_f64* xc0, lds_f64* xc1, lds_f64* pv, lds_f64* red, gbl_f64* refl) {
  const int tid = threadIdx.x;
  const int br = tid >> 4, bc = tid & 15, lane = tid & 63, wave = tid >> 6;
  double a[8][8];
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int r = 8 * br + q, s2 = 8 * bc + c;
      a[q][c] = (r < n && s2 < n) ? H[r * n + s2] : 0.0;
    }
  lds_f64* kpart = red + 32;  // [4] partial v^T p, per wavefront
  // the column and p live in LDS with element 8 b + q in slot 16 q + b, so that
  // the 16 lanes of a row (b = bc) read 16 consecutive words
  auto slot = [](int r) { return (r & 7) * 16 + (r >> 3); };
  const int tri_tid = tri(tid);
  // column i of the current matrix, as held by its owners (bc == i / 8); taken
  // inside a statically unrolled column loop under a uniform condition
  double xo[8];
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (c == 0) {
#pragma unroll
      for (int q = 0; q < 8; ++q) xo[q] = a[q][c];
    }
  for (int i = 0; i < n - 2; ++i) {
    lds_f64* xcol = (i & 1) ? xc1 : xc0;        // column i
    lds_f64* nrm = red + 16 * (i & 1);          // [16] its partial norms, per block row
    const bool owner = bc == (i >> 3);
    if (owner) {
      double s2 = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        xcol[16 * q + br] = xo[q];
        if (8 * br + q >= i + 2) s2 += xo[q] * xo[q];
      }
      nrm[br] = s2;
    }
    __syncthreads();
    // every thread forms the reflector (dlarfg): beta = -sign(alpha) |(alpha, x)|
    const double alpha = xcol[slot(i + 1)];
    double xn2 = 0.0;
#pragma unroll
    for (int b = 0; b < 16; ++b) xn2 += nrm[b];
    double beta = alpha, t = 0.0, scal = 0.0;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (tid == 0) { dg[i] = xcol[slot(i)]; eg[i] = beta; tau[i] = t; }
    if (tid > i && tid < n)  // reflector entry of row tid, from the published column
      refl[tri_tid + i] = (tid == i + 1) ? 1.0 : (double)xcol[slot(tid)] * scal;
    if (t != 0.0) {  // uniform
      // all 16 column entries are read before any is used (every slot holds a
      // value: rows beyond n are zero), so the reads overlap
      double xcv[8], xrv[8], vc[8], vr[8], pr[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        xcv[q] = xcol[16 * q + bc];
        xrv[q] = xcol[16 * q + br];
      }
      // v on the tile's columns and rows: 1 at row i + 1, x scal beyond it up
      // to n, 0 elsewhere (selects, no branches); indices relative to the tile
      const int uc = i + 1 - 8 * bc, nc = n - 8 * bc, ur = i + 1 - 8 * br, nr = n - 8 * br;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double xc = xcv[q] * scal, xr = xrv[q] * scal;
        vc[q] = ((q > uc) & (q < nc)) ? xc : 0.0;
        vr[q] = ((q > ur) & (q < nr)) ? xr : 0.0;
        vc[q] = q == uc ? 1.0 : vc[q];
        vr[q] = q == ur ? 1.0 : vr[q];
      }
      // the eight row products advance together, then their sums over the 16
      // lanes of the row stage by stage (quad_perm [1,0,3,2] and [2,3,0,1] sum
      // each quad, row_half_mirror pairs the quads of each half, row_mirror the
      // halves), so that consecutive instructions are independent
#pragma unroll
      for (int q = 0; q < 8; ++q) pr[q] = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int q = 0; q < 8; ++q) pr[q] += a[q][c] * vc[c];
#pragma unroll
      for (int q = 0; q < 8; ++q) pr[q] += dpp_f64<0xB1>(pr[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q) pr[q] += dpp_f64<0x4E>(pr[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q) pr[q] += dpp_f64<0x141>(pr[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q) pr[q] += dpp_f64<0x140>(pr[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q) pr[q] *= t;
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) part += pr[q] * vr[q];
      // v^T p: four block rows per wavefront, then across wavefronts
      part = xor32_sum(xor16_sum(part));
      if (bc == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) pv[16 * q + br] = pr[q];
      }
      if (lane == 0) kpart[wave] = part;
      __syncthreads();
      const double K = -0.5 * t * (((double)kpart[0] + (double)kpart[1]) + ((double)kpart[2] + (double)kpart[3]));
#pragma unroll
      for (int q = 0; q < 8; ++q) pr[q] += K * vr[q];  // w on the tile's rows
      const int cn = (i + 1) & 7;  // column of the next step within its tile
      double pc[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) pc[c] = pv[16 * c + bc];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const double wc = pc[c] + K * vc[c];  // w on the tile's columns
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q][c] = fma(-pr[q], vc[c], fma(-vr[q], wc, a[q][c]));
        if (c == cn) {
#pragma unroll
          for (int q = 0; q < 8; ++q) xo[q] = a[q][c];
        }
      }
    } else {
      const int cn = (i + 1) & 7;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c == cn) {
#pragma unroll
          for (int q = 0; q < 8; ++q) xo[q] = a[q][c];
        }
    }
    // next step: its column goes to the other buffer; pv and kpart are written
    // only after its first barrier, which every thread reaches after its reads above
  }
  // the last 2 x 2 block
  if (n >= 2) {
    const int i0 = n - 2, i1 = n - 1;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int r = 8 * br + q, s2 = 8 * bc + c;
        if (r == i0 && s2 == i0) dg[i0] = a[q][c];
        if (r == i1 && s2 == i0) eg[i0] = a[q][c];
        if (r == i1 && s2 == i1) dg[i1] = a[q][c];
      }
    if (tid == 0) { tau[i0] = 0.0; eg[i1] = 0.0; tau[i1] = 0.0; }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (8 * br + q == 0 && 8 * bc + c == 0) dg[0] = a[q][c];
    if (tid == 0) { eg[0] = 0.0; tau[0] = 0.0; }
  }
  __syncthreads();
}

// H: n x n symmetric, row-major (ld n), in global memory; n <= EIG_NMAX.
// Writes the eigenvectors of the k largest eigenvalues, in descending order,
// as columns 0..k-1 of V (ld k) and the eigenvalues to lam[0..k-1].
// refl: global scratch of at least EIG_PACK doubles (Householder vectors);
// lds: EIG_LDS_BYTES of LDS owned by the caller.
__device__ __forceinline__ void sym_topk_eig(const double* H, int n, int k, double* V, double* lam, double* refl, char* lds) {
  double* Ap = reinterpret_cast<double*>(lds);
  double* Xs = Ap + 3 * EIG_NMAX * EIG_KMAX;                            // after the tridiagonalisation
  double* dg = reinterpret_cast<double*>(lds + EIG_PACK_BYTES);
  double* eg = dg + EIG_NMAX;
  double* e2 = eg + EIG_NMAX;
  double* tau = e2 + EIG_NMAX;
  double* pv = tau + EIG_NMAX;
  double* wv = pv + EIG_NMAX;
  double* vv = wv + EIG_NMAX;
  double* probe_x = vv + 3 * EIG_NMAX;
  double* lamb = probe_x + WG;
  const int tid = threadIdx.x;

  // ---- tridiagonalisation (out of line: its register tile needs the whole register budget)
  eig_tridiag((const gbl_f64*)H, n, (lds_f64*)(dg), (lds_f64*)(eg), (lds_f64*)(tau), (lds_f64*)(wv),
              (lds_f64*)(vv), (lds_f64*)(pv), (lds_f64*)(probe_x), (gbl_f64*)refl);
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
    // A group's 16 lanes lie in one wavefront: the first probe with more than
    // q eigenvalues below it is found by a ballot, and the new interval's ends
    // are read from its lane and the lane before (no LDS, no barrier).
    const int gl = (tid & 63) & ~15;  // lane 0 of this group within the wavefront
    for (int it = 0; it < 13; ++it) {  // 17^13 > 2^52
      const double x = a + (c - a) * (double)(lane + 1) / 17.0;
      const int cnt = (g < kb) ? sturm_count(dg, e2, n, x, pivmin) : 0;
      const unsigned long long above = __ballot(cnt > q);
      const unsigned gm = (unsigned)(above >> gl) & 0xFFFFu;
      const int s1 = gm ? __builtin_ctz(gm) : 16;  // probes 0 .. s1-1 have at most q below them
      const double xl = __shfl(x, gl + max(s1 - 1, 0), 64);
      const double xh = __shfl(x, gl + min(s1, 15), 64);
      if (g < kb) {
        if (s1 > 0) a = xl;
        if (s1 < 16) c = xh;
      }
    }
    if (g < kb && lane == 0) lamb[g] = 0.5 * (a + c);
    // deterministic, eigenvector-dependent start vectors: entry j of vector t
    // at Xs[j * EIG_KMAX + t], written by the whole work-group
    for (int e = tid; e < n * EIG_KMAX; e += WG) {
      const int j = e / EIG_KMAX, t = e - j * EIG_KMAX;
      if (t < kb) {
        uint64_t h = (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull ^ (uint64_t)(b0 + t + 1) * 0xD2E7470EE14C6C93ull;
        h ^= h >> 29;
        Xs[e] = 0.5 + (double)(h & 0xFFFF) / 65536.0;
      }
    }
    __syncthreads();

    // ---- inverse iteration, one thread per eigenvector; LU factors in LDS (Ap is free now)
    double* U0 = Ap;                               // reciprocal pivots
    double* U1 = Ap + 1 * EIG_NMAX * EIG_KMAX;     // first superdiagonal of U
    double* ML = Ap + 2 * EIG_NMAX * EIG_KMAX;     // multipliers
    double* inv_nrm = probe_x;                     // per vector: 1 / max |x| of the last iterate
    if (tid < kb) {
      const double lm = lamb[tid];
      const int nm1 = n - 1;  // elimination steps
#define IX(j) ((j) * EIG_KMAX + tid)
      // Steps run in blocks of four whose operands are read one block ahead;
      // the row swaps are kept as bits in registers (bit j % 32 of word j / 32).
      unsigned pb[EIG_NMAX / 32] = {0u, 0u, 0u, 0u};
      auto word = [&](int j) {
        const int w = j >> 5;
        return w == 0 ? pb[0] : (w == 1 ? pb[1] : (w == 2 ? pb[2] : pb[3]));
      };
      // Gaussian elimination with partial pivoting of T - lm I; a swap of rows j
      // and j+1 puts the known entry e[j+1] on the second superdiagonal.
      double aa = dg[0] - lm, cc = n > 1 ? eg[0] : 0.0, bb = cc;  // bb = e_j
      double nd[4], ne[4];  // d_{j+1}, e_{j+1} of the next block
#pragma unroll
      for (int q = 0; q < 4; ++q) { nd[q] = dg[min(q + 1, n - 1)]; ne[q] = eg[min(q + 1, n - 1)]; }
      for (int jb = 0; jb < nm1; jb += 4) {
        double cd[4], ce[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          cd[q] = nd[q]; ce[q] = ne[q];
          nd[q] = dg[min(jb + 5 + q, n - 1)];
          ne[q] = eg[min(jb + 5 + q, n - 1)];
        }
        unsigned bits = 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = jb + q;
          if (j < nm1) {
            const double a1 = cd[q] - lm;
            const double c1 = (j + 1 < nm1) ? ce[q] : 0.0;
            // no swap: pivot aa (kept away from zero), U row (aa, cc), next row
            // (a1 - m cc, c1); swap: pivot bb, U row (bb, a1, e[j+1]), next row
            // (cc - m a1, -m c1).  Both by selects, so the lanes do not diverge.
            const bool sw = fabs(aa) < fabs(bb);
            const double pa = fabs(aa) < tiny ? (aa < 0.0 ? -tiny : tiny) : aa;
            const double ip = recip(sw ? bb : pa);
            const double m = (sw ? aa : bb) * ip;
            const double u1 = sw ? a1 : cc;
            U0[IX(j)] = ip; U1[IX(j)] = u1; ML[IX(j)] = m;
            bits |= (sw ? 1u : 0u) << q;
            aa = fma(-m, u1, sw ? cc : a1);
            cc = sw ? -m * c1 : c1;
            bb = c1;
          }
        }
        const int w = jb >> 5;
#pragma unroll
        for (int i = 0; i < EIG_NMAX / 32; ++i) pb[i] |= (w == i) ? bits << (jb & 31) : 0u;
      }
      U0[IX(nm1)] = recip(fabs(aa) < tiny ? (aa < 0.0 ? -tiny : tiny) : aa);
      U1[IX(nm1)] = 0.0;  // the last row has no superdiagonal
      double s = 1.0;     // scale of the current iterate, applied as it is read
      for (int it = 0; it < EIG_INV_ITERS; ++it) {
        // forward elimination; the running entry j + 1 stays in a register
        double carry = Xs[IX(0)] * s;
        double nx[4], nm[4];  // Xs[j+1], ML[j] of the next block
#pragma unroll
        for (int q = 0; q < 4; ++q) { nx[q] = Xs[IX(min(q + 1, nm1))]; nm[q] = ML[IX(min(q, nm1))]; }
        for (int jb = 0; jb < nm1; jb += 4) {
          double cx[4], cm[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            cx[q] = nx[q]; cm[q] = nm[q];
            nx[q] = Xs[IX(min(jb + 5 + q, nm1))];
            nm[q] = ML[IX(min(jb + 4 + q, nm1))];
          }
          const unsigned bits = word(jb) >> (jb & 31);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = jb + q;
            if (j < nm1) {
              double rj = carry, rj1 = cx[q] * s;
              if ((bits >> q) & 1u) { const double tt = rj; rj = rj1; rj1 = tt; }
              Xs[IX(j)] = rj;
              carry = rj1 - cm[q] * rj;
            }
          }
        }
        Xs[IX(nm1)] = carry;
        // back substitution from row n - 1 down, in blocks of four rows
        double x1 = 0.0, x2 = 0.0, nrm = 0.0;
        double px[4], pu1[4], pu0[4], pe[4];  // rows jt - q of the next block
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = max(nm1 - q, 0);
          px[q] = Xs[IX(j)]; pu1[q] = U1[IX(j)]; pu0[q] = U0[IX(j)]; pe[q] = eg[min(j + 1, nm1)];
        }
        for (int jt = nm1; jt >= 0; jt -= 4) {
          double cx[4], cu1[4], cu0[4], ce[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            cx[q] = px[q]; cu1[q] = pu1[q]; cu0[q] = pu0[q]; ce[q] = pe[q];
            const int j = max(jt - 4 - q, 0);
            px[q] = Xs[IX(j)]; pu1[q] = U1[IX(j)]; pu0[q] = U0[IX(j)]; pe[q] = eg[min(j + 1, nm1)];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = jt - q;
            if (j >= 0) {
              const bool swp = (word(j) >> (j & 31)) & 1u;
              const double u2 = (swp && j + 1 < nm1) ? ce[q] : 0.0;
              const double xj = (cx[q] - cu1[q] * x1 - u2 * x2) * cu0[q];  // U0 holds 1/pivot
              Xs[IX(j)] = xj;
              x2 = x1;
              x1 = xj;
              nrm = fmax(nrm, fabs(xj));
            }
          }
        }
        s = nrm > 0.0 ? 1.0 / nrm : 1.0;
      }
      inv_nrm[tid] = s;
#undef IX
    }
    __syncthreads();
    // the last iterate's scale, applied by the whole work-group
    for (int e = tid; e < n * EIG_KMAX; e += WG) {
      const int t = e % EIG_KMAX;
      if (t < kb) Xs[e] *= inv_nrm[t];
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

  // ---- classical Gram-Schmidt, twice, over the kept vectors in descending
  // order; each vector is brought to unit norm as soon as it is orthogonalised,
  // so that the projections of the later vectors onto it are exact projections
  // (inverse iteration leaves the vectors scaled to max |x| = 1, not to unit
  // norm).  Vw is the LDS or the global copy of the vectors.
  auto orthonormalise = [&](auto* Vw, int ld) {
    auto unit = [&](int col) {
      double nn = 0.0;
      for (int j = tid; j < n; j += WG) nn += Vw[j * ld + col] * Vw[j * ld + col];
      nn = wg_sum(nn);
      const double f = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int j = tid; j < n; j += WG) Vw[j * ld + col] *= f;
      __syncthreads();
    };
    unit(0);
    for (int col = 1; col < k; ++col) {
      for (int pass = 0; pass < 2; ++pass) {
        // dots with every earlier (unit) vector: 16 lanes per earlier vector
        for (int s0 = 0; s0 < col; s0 += WG / 16) {
          const int sv = s0 + (tid >> 4);
          double dp = 0.0;
          if (sv < col)
            for (int j = tid & 15; j < n; j += 16) dp += Vw[j * ld + sv] * Vw[j * ld + col];
          dp = row16_sum(dp);
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
      unit(col);
    }
  };
  const gbl_f64* rf = (const gbl_f64*)refl;
  // entry tid of reflector i (zero outside rows i + 1 .. n - 1)
  auto refl_entry = [&](int i) -> double { return (tid > i && tid < n) ? rf[tri(tid) + i] : 0.0; };

  // ---- back-transformation: x <- H_0 H_1 ... H_{n-3} x
  if (in_lds) {
    orthonormalise((lds_f64*)Xs, EIG_KMAX);
    // the k <= 16 vectors in registers: thread t holds rows 8 (t / 16) .. +7 of
    // column t % 16; reflector i is staged in one of two LDS rows while the
    // previous one is applied (read from global memory one step before it is
    // staged), and the column sums of v^T x alternate between two LDS rows, so
    // one barrier per reflector suffices.
    const int col = tid & 15, rb = tid >> 4, wave = tid >> 6;
    lds_f64* const vb0 = (lds_f64*)vv;
    lds_f64* const vb1 = (lds_f64*)wv;
    lds_f64* const rs0 = (lds_f64*)pv;       // [4 waves][16 columns] each
    lds_f64* const rs1 = (lds_f64*)probe_x;
    const lds_f64* xl = (const lds_f64*)Xs;
    double x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = 8 * rb + q;
      x[q] = (r < n && col < k) ? xl[r * EIG_KMAX + col] : 0.0;
    }
    if (n >= 3 && tid < EIG_NMAX) (((n - 3) & 1) ? vb1 : vb0)[tid] = refl_entry(n - 3);
    double vnext = (n >= 4 && tid < EIG_NMAX) ? refl_entry(n - 4) : 0.0;
    __syncthreads();
    for (int i = n - 3; i >= 0; --i) {
      const lds_f64* v = (i & 1) ? vb1 : vb0;
      double vr[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) vr[q] = v[8 * rb + q];
      const double t = tau[i];
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) part += vr[q] * x[q];
      part = xor32_sum(xor16_sum(part));
      lds_f64* red = (i & 1) ? rs1 : rs0;
      if ((tid & 63) < 16) red[wave * 16 + col] = part;
      // stage reflector i - 1 (every reader of that row has passed the previous
      // barrier) and read reflector i - 2
      if (i >= 1 && tid < EIG_NMAX) (((i - 1) & 1) ? vb1 : vb0)[tid] = vnext;
      if (i >= 2 && tid < EIG_NMAX) vnext = refl_entry(i - 2);
      __syncthreads();
      const double f = t * ((red[col] + red[16 + col]) + (red[32 + col] + red[48 + col]));
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] -= f * vr[q];
    }
    gbl_f64* Vg = (gbl_f64*)V;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = 8 * rb + q;
      if (r < n && col < k) Vg[(int64_t)r * k + col] = x[q];
    }
    __syncthreads();
    return;
  }
  // more than 16 vectors, in V: reflector i staged in LDS, the next one read
  // into a register while the current one is applied
  gbl_f64* Vg = (gbl_f64*)V;
  orthonormalise(Vg, k);
  double vreg = (n >= 3 && tid < EIG_NMAX) ? refl_entry(n - 3) : 0.0;
  for (int i = n - 3; i >= 0; --i) {
    if (tid < n) vv[tid] = vreg;
    if (i >= 1 && tid < EIG_NMAX) vreg = refl_entry(i - 1);
    __syncthreads();
    const double t = tau[i];
    if (t != 0.0) {
      for (int c0 = 0; c0 < k; c0 += WG / 16) {
        const int col = c0 + (tid >> 4);
        double dp = 0.0;
        if (col < k)
          for (int r = i + 1 + (tid & 15); r < n; r += 16) dp += vv[r] * Vg[r * k + col];
        dp = row16_sum(dp);
        if ((tid & 15) == 0 && col < k) pv[col] = t * dp;
      }
      __syncthreads();
      for (int e = tid; e < (n - i - 1) * k; e += WG) {
        const int rr = e / k, col = e - rr * k;
        const int r = i + 1 + rr;
        Vg[r * k + col] -= pv[col] * vv[r];
      }
    }
    __syncthreads();
  }
}

}  // namespace vp
