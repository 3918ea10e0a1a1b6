// Simple-update imaginary-time evolution (App. A), nearest-neighbour terms.
//
// The PEPS is held as site tensors B (the canonical flat layout of the
// parameters) and a diagonal matrix lambda on every link (D numbers per link:
// horizontal links (y,x)-(y,x+1) first, row-major, then vertical links
// (y,x)-(y+1,x)).  A step applies exp(-dt J S_A.S_B) once to every link, in
// four classes: horizontal links with x even, with x odd, vertical links with
// y even, with y odd.  Links of one class share no site, so one work-group per
// link updates a class in any order with the same result.  Per link (App. A,
// Fig. 8 (b)-(h), two sites):
//   1. the lambdas of the outer links multiply both site tensors, written as
//      matrices X = (outer legs) x (s, bond);
//   2. thin Householder QR of each (when it has more rows than columns):
//      X_A = Q_A R_A, X_B = Q_B R_B;
//   3. Theta[(a, t_A), (t_B, b)] = sum G[t_A t_B; s_A s_B] R_A[a, (s_A, k)]
//      lambda_k R_B[b, (s_B, k)] with the exact bond gate G;
//   4. the leading singular triplets of Theta from the eigenproblem of
//      Theta Theta^T (the compression's float64 eigensolver): U, sigma, and
//      V^T = sigma^-1 U^T Theta; sigma below 1e-6 sigma_1 is dropped, the kept
//      ones normalised to unit 2-norm become the link's lambda;
//   5. the new tensors Q_A U and Q_B V with the outer lambdas divided out
//      (1/lambda where lambda > 0, else 0).
// Next-nearest-neighbour terms (both diagonals of every plaquette) follow
// Fig. 8: the pair (B_1, B_3) is joined through a corner site B_2 (the
// diagonal (y,x)-(y+1,x+1) through (y,x+1), the anti-diagonal (y,x+1)-(y+1,x)
// through (y,x)); B_1 and B_3 are QR-reduced, the gate acts on the reduced
// three-site tensor T_a = R_1 lambda_4 B_2 lambda_7 R_3^T, a truncated SVD
// gives R~_1 and lambda~_4, a second one of lambda~_4 T_b gives T_c, lambda~_7
// and R~_3, and B_2 = T_c / lambda~_4.  Plaquettes go in four classes
// (y mod 2, x mod 2), diagonals then anti-diagonals, after the
// nearest-neighbour classes; plaquettes of one class share no site.
// All of it in float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "vp_fit.hpp"
#include "vp_kernels.hpp"

namespace vp {

namespace {

constexpr double SU_DROP = 1e-6;

struct SuArgs {
  double* B;            // site tensors, canonical flat layout
  double* lam;          // [n_links][D]
  const int64_t* offs;  // [N+1]
  const int32_t* dims;  // [N][4] (l, u, r, d)
  int Ly, Lx, D;
  int cls;              // link class 0..3
  int first;            // first link of the class handled by this launch
  double dt, J;
  double* scr;          // per work-group scratch
  int64_t scr_stride;
  double* unused;
};

__device__ inline int link_h(const SuArgs& a, int y, int x) { return y * (a.Lx - 1) + x; }
__device__ inline int link_v(const SuArgs& a, int y, int x) { return a.Ly * (a.Lx - 1) + y * a.Lx + x; }

// Link of leg q (0 l, 1 u, 2 r, 3 d) of site (y, x), or -1 on the open boundary.
__device__ inline int leg_link(const SuArgs& a, int y, int x, int q) {
  if (q == 0) return x > 0 ? link_h(a, y, x - 1) : -1;
  if (q == 1) return y > 0 ? link_v(a, y - 1, x) : -1;
  if (q == 2) return x < a.Lx - 1 ? link_h(a, y, x) : -1;
  return y < a.Ly - 1 ? link_v(a, y, x) : -1;
}

__device__ inline double pinv(double v) { return v > 0.0 ? 1.0 / v : 0.0; }

// One site of the link: its outer legs (increasing leg order) and their extents.
struct SuSite {
  int y, x, k, bond_leg;
  int d[4];
  int o[3];      // outer legs
  int olink[3];  // their links (-1: open boundary)
  int m;         // product of the outer extents
  int64_t base;  // offset of the site in B
  int size;      // l u r d
};

__device__ inline SuSite su_site(const SuArgs& a, int y, int x, int bond_leg) {
  SuSite s;
  s.y = y; s.x = x; s.k = y * a.Lx + x; s.bond_leg = bond_leg;
  for (int q = 0; q < 4; ++q) s.d[q] = a.dims[4 * s.k + q];
  int j = 0;
  for (int q = 0; q < 4; ++q)
    if (q != bond_leg) { s.o[j] = q; s.olink[j] = leg_link(a, y, x, q); ++j; }
  s.m = s.d[s.o[0]] * s.d[s.o[1]] * s.d[s.o[2]];
  s.base = a.offs[s.k];
  s.size = s.d[0] * s.d[1] * s.d[2] * s.d[3];
  return s;
}

// Offset within one physical slice of the element with outer row o and bond index k,
// and the product of the outer lambdas at that element (or of their inverses).
__device__ inline int su_addr(const SuArgs& a, const SuSite& s, int o, int k, double* lam_prod, bool inverse) {
  int idx[4];
  const int e2 = s.d[s.o[2]], e1 = s.d[s.o[1]];
  idx[s.o[2]] = o % e2;
  idx[s.o[1]] = (o / e2) % e1;
  idx[s.o[0]] = o / (e2 * e1);
  idx[s.bond_leg] = k;
  double p = 1.0;
  for (int j = 0; j < 3; ++j)
    if (s.olink[j] >= 0) {
      const double l = a.lam[(int64_t)s.olink[j] * a.D + idx[s.o[j]]];
      p *= inverse ? pinv(l) : l;
    }
  *lam_prod = p;
  return ((idx[0] * s.d[1] + idx[1]) * s.d[2] + idx[2]) * s.d[3] + idx[3];
}

// Gate exp(-dt J S_A.S_B) element G[t_A t_B; s_A s_B] (s = 0 is S^z = +1/2):
// exp(-dt J / 4) on the triplet, exp(3 dt J / 4) on the singlet.
__device__ inline double su_gate(double ga, double gb, int tA, int tB, int sA, int sB) {
  if (tA + tB != sA + sB) return 0.0;                 // S^z conserved
  if (tA == tB) return ga;                            // |uu>, |dd>
  return tA == sA ? 0.5 * (ga + gb) : 0.5 * (ga - gb);  // antiparallel block
}

// LDS of one link update: the eigensolver's.
constexpr size_t SU_LDS = EIG_LDS_BYTES;

__global__ void __launch_bounds__(WG) k_su_link(SuArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[SU_LDS];
  __shared__ int s_kk;
  const int tid = threadIdx.x;
  // the link of this work-group
  const int bidx = a.first + blockIdx.x;
  const bool horiz = a.cls < 2;
  int y, x;
  if (horiz) {
    const int per_row = a.cls == 0 ? a.Lx / 2 : (a.Lx - 1) / 2;
    y = bidx / per_row;
    x = 2 * (bidx % per_row) + a.cls;
  } else {
    y = 2 * (bidx / a.Lx) + (a.cls - 2);
    x = bidx % a.Lx;
  }
  const int link = horiz ? link_h(a, y, x) : link_v(a, y, x);
  const SuSite A = su_site(a, y, x, horiz ? 2 : 3);
  const SuSite Bs = horiz ? su_site(a, y, x + 1, 0) : su_site(a, y + 1, x, 1);
  const int kd = A.d[A.bond_leg];  // the link's extent (= D)
  const int n = 2 * kd;            // columns (s, k) of X
  const int M = a.D * a.D * a.D;   // the largest outer extent
  double* w = a.scr + (int64_t)blockIdx.x * a.scr_stride;
  double* XA = w;                  // M n: X_A, then Q_A
  double* XB = XA + (int64_t)M * n;
  double* Xs = XB + (int64_t)M * n;  // QR scratch
  double* Qs = Xs + (int64_t)M * n;
  double* RA = Qs + (int64_t)M * n;  // n x n
  double* RB = RA + n * n;
  double* Th = RB + n * n;           // (2n) x (2n)
  double* H = Th + 4 * n * n;        // (2n) x (2n)
  double* U = H + 4 * n * n;         // (2n) x kd
  double* Vt = U + 2 * n * kd;       // kd x (2n)
  double* ev = Vt + 2 * n * kd;      // 64
  double* refl = ev + 64;            // EIG_PACK
  const double* lam_bond = a.lam + (int64_t)link * a.D;

  // 1. X = (outer) x (s, k) with the outer lambdas multiplied in
  for (int e = tid; e < A.m * n; e += WG) {
    const int o = e % A.m, c = e / A.m, s = c / kd, k = c % kd;
    double lp;
    const int off = su_addr(a, A, o, k, &lp, false);
    XA[e] = a.B[A.base + (int64_t)s * A.size + off] * lp;
  }
  for (int e = tid; e < Bs.m * n; e += WG) {
    const int o = e % Bs.m, c = e / Bs.m, s = c / kd, k = c % kd;
    double lp;
    const int off = su_addr(a, Bs, o, k, &lp, false);
    XB[e] = a.B[Bs.base + (int64_t)s * Bs.size + off] * lp;
  }
  __syncthreads();
  // 2. reduced tensors R (rows a < r, columns (s, k)); Q stays in X when the QR is taken
  const bool qrA = A.m > n, qrB = Bs.m > n;
  const int rA = qrA ? n : A.m, rB = qrB ? n : Bs.m;
  if (qrA) {
    fit_qr<double>(XA, A.m * n, colmajor(A.m), A.m, n, Xs, Qs);
    for (int e = tid; e < n * n; e += WG) {
      const int r = e / n, c = e % n;
      RA[e] = r <= c ? Xs[r + (int64_t)c * A.m] : 0.0;
    }
  } else {
    for (int e = tid; e < rA * n; e += WG) RA[e] = XA[(e / n) + (int64_t)(e % n) * A.m];
  }
  __syncthreads();
  if (qrB) {
    fit_qr<double>(XB, Bs.m * n, colmajor(Bs.m), Bs.m, n, Xs, Qs);
    for (int e = tid; e < n * n; e += WG) {
      const int r = e / n, c = e % n;
      RB[e] = r <= c ? Xs[r + (int64_t)c * Bs.m] : 0.0;
    }
  } else {
    for (int e = tid; e < rB * n; e += WG) RB[e] = XB[(e / n) + (int64_t)(e % n) * Bs.m];
  }
  __syncthreads();
  // 3. Theta with the gate, rows (a, t_A) and columns (t_B, b)
  const double ga = exp(-0.25 * a.dt * a.J), gb = exp(0.75 * a.dt * a.J);
  const int R = 2 * rA, C = 2 * rB;
  for (int e = tid; e < rA * rB; e += WG) {
    const int ia = e / rB, ib = e % rB;
    double P[2][2];
    for (int sA = 0; sA < 2; ++sA)
      for (int sB = 0; sB < 2; ++sB) {
        double acc = 0.0;
        for (int k = 0; k < kd; ++k) acc += RA[ia * n + sA * kd + k] * lam_bond[k] * RB[ib * n + sB * kd + k];
        P[sA][sB] = acc;
      }
    for (int tA = 0; tA < 2; ++tA)
      for (int tB = 0; tB < 2; ++tB) {
        double v = 0.0;
        for (int sA = 0; sA < 2; ++sA)
          for (int sB = 0; sB < 2; ++sB) v += su_gate(ga, gb, tA, tB, sA, sB) * P[sA][sB];
        Th[(ia * 2 + tA) * C + tB * rB + ib] = v;
      }
  }
  __syncthreads();
  // 4. the kept singular triplets
  for (int e = tid; e < R * R; e += WG) {
    const int i = e / R, j = e % R;
    double acc = 0.0;
    for (int c = 0; c < C; ++c) acc += Th[i * C + c] * Th[j * C + c];
    H[e] = acc;
  }
  __syncthreads();
  const int kk0 = min(kd, min(R, C));
  sym_topk_eig(H, R, kk0, U, ev, refl, lds);
  if (tid == 0) {
    const double s0 = sqrt(fmax(ev[0], 0.0));
    int kk = 0;
    if (s0 > 0.0)
      while (kk < kk0 && sqrt(fmax(ev[kk], 0.0)) > SU_DROP * s0) ++kk;
    s_kk = kk;
  }
  __syncthreads();
  const int kk = s_kk;
  double nrm2 = 0.0;
  for (int i = 0; i < kk; ++i) nrm2 += fmax(ev[i], 0.0);
  const double inv_nrm = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
  // V^T = sigma^-1 U^T Theta (rows i < kk), zero beyond
  for (int e = tid; e < kd * C; e += WG) {
    const int i = e / C, c = e % C;
    double v = 0.0;
    if (i < kk) {
      for (int r = 0; r < R; ++r) v += U[r * kk0 + i] * Th[r * C + c];
      v /= sqrt(fmax(ev[i], 0.0));
    }
    Vt[e] = v;
  }
  __syncthreads();
  // 5. new site tensors: Q_A U and Q_B V, outer lambdas divided out
  for (int e = tid; e < A.m * n; e += WG) {
    const int o = e % A.m, c = e / A.m, t = c / kd, i = c % kd;
    double v = 0.0;
    if (i < kk) {
      if (qrA)
        for (int r = 0; r < rA; ++r) v += XA[o + (int64_t)r * A.m] * U[(r * 2 + t) * kk0 + i];
      else
        v = U[(o * 2 + t) * kk0 + i];
    }
    double ip;
    const int off = su_addr(a, A, o, i, &ip, true);
    a.B[A.base + (int64_t)t * A.size + off] = v * ip;
  }
  for (int e = tid; e < Bs.m * n; e += WG) {
    const int o = e % Bs.m, c = e / Bs.m, t = c / kd, i = c % kd;
    double v = 0.0;
    if (i < kk) {
      if (qrB)
        for (int r = 0; r < rB; ++r) v += XB[o + (int64_t)r * Bs.m] * Vt[i * C + t * rB + r];
      else
        v = Vt[i * C + t * rB + o];
    }
    double ip;
    const int off = su_addr(a, Bs, o, i, &ip, true);
    a.B[Bs.base + (int64_t)t * Bs.size + off] = v * ip;
  }
  // the link's new lambda (every thread has read the old one)
  __syncthreads();
  if (tid < kd) a.lam[(int64_t)link * a.D + tid] = tid < kk ? sqrt(fmax(ev[tid], 0.0)) * inv_nrm : 0.0;
}

// The leading singular triplets of a matrix from the eigenproblem of its Gram
// matrix H (R x R, already formed): U (R x k0, ld k0), eigenvalues ev; returns
// the kept count (sigma > SU_DROP sigma_1) and 1 / the 2-norm of the kept sigmas.
__device__ inline int su_top(double* H, int R, int k0, double* U, double* ev, double* refl, char* lds, int* s_kk,
                             double* inv_nrm) {
  sym_topk_eig(H, R, k0, U, ev, refl, lds);
  if (threadIdx.x == 0) {
    const double s0 = sqrt(fmax(ev[0], 0.0));
    int kk = 0;
    if (s0 > 0.0)
      while (kk < k0 && sqrt(fmax(ev[kk], 0.0)) > SU_DROP * s0) ++kk;
    *s_kk = kk;
  }
  __syncthreads();
  const int kk = *s_kk;
  double nrm2 = 0.0;
  for (int i = 0; i < kk; ++i) nrm2 += fmax(ev[i], 0.0);
  *inv_nrm = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
  return kk;
}

// The X = (outer) x (s, bond) matrix of one end site with its outer lambdas,
// QR-reduced when it has more rows than columns: R (r x n, row-major) and Q
// left in X.  Returns r.
__device__ inline int su_reduce(const SuArgs& a, const SuSite& S, double* X, double* R, int kd, double* Xs,
                                double* Qs) {
  const int n = 2 * kd;
  for (int e = threadIdx.x; e < S.m * n; e += WG) {
    const int o = e % S.m, c = e / S.m, s = c / kd, k = c % kd;
    double lp;
    const int off = su_addr(a, S, o, k, &lp, false);
    X[e] = a.B[S.base + (int64_t)s * S.size + off] * lp;
  }
  __syncthreads();
  if (S.m > n) {
    fit_qr<double>(X, S.m * n, colmajor(S.m), S.m, n, Xs, Qs);
    for (int e = threadIdx.x; e < n * n; e += WG) {
      const int r = e / n, c = e % n;
      R[e] = r <= c ? Xs[r + (int64_t)c * S.m] : 0.0;
    }
    __syncthreads();
    return n;
  }
  for (int e = threadIdx.x; e < S.m * n; e += WG) R[e] = X[(e / n) + (int64_t)(e % n) * S.m];
  __syncthreads();
  return S.m;
}

// Scratch of one three-site update (doubles) and its regions.
__host__ __device__ inline int64_t su_nnn_doubles(int D) {
  const int64_t n = 2 * D, M = (int64_t)D * D * D, D2 = (int64_t)D * D;
  return 4 * M * n + 2 * n * n + 2 * D2 * D2 + 2 * (4 * n * D * D2) + 8 * n * n * D2 + 2 * 4 * n * n +
         2 * 2 * n * D + 2 * D2 * D2 + 128 + EIG_PACK;
}

// One next-nearest-neighbour pair per work-group: plaquette first + blockIdx.x of class a.cls (0..3),
// the anti-diagonal when `anti`.
__global__ void __launch_bounds__(WG) k_su_nnn(SuArgs a, int anti) {
  __shared__ __attribute__((aligned(16))) char lds[SU_LDS];
  __shared__ int s_kk;
  const int tid = threadIdx.x;
  const int py = a.cls >> 1, px = a.cls & 1;
  const int nx = (a.Lx - px) / 2;
  const int b = a.first + blockIdx.x;
  const int y = py + 2 * (b / nx), x = px + 2 * (b % nx);
  // B_1 -(link 4)- B_2 -(link 7)- B_3
  const SuSite S1 = anti ? su_site(a, y, x + 1, 0) : su_site(a, y, x, 2);
  const SuSite S3 = anti ? su_site(a, y + 1, x, 1) : su_site(a, y + 1, x + 1, 1);
  const int y2 = y, x2 = anti ? x : x + 1;
  const int l21 = anti ? 2 : 0, l23 = 3;
  const int k2 = y2 * a.Lx + x2;
  int d2[4];
  for (int q = 0; q < 4; ++q) d2[q] = a.dims[4 * k2 + q];
  int o2[2], o2link[2], j2 = 0;
  for (int q = 0; q < 4; ++q)
    if (q != l21 && q != l23) { o2[j2] = q; o2link[j2] = leg_link(a, y2, x2, q); ++j2; }
  const int n2 = d2[o2[0]] * d2[o2[1]];
  const int64_t base2 = a.offs[k2];
  const int size2 = d2[0] * d2[1] * d2[2] * d2[3];
  const int link4 = leg_link(a, S1.y, S1.x, S1.bond_leg), link7 = leg_link(a, S3.y, S3.x, S3.bond_leg);
  const int D = a.D, n = 2 * D, M = D * D * D, D2 = D * D;
  double* w = a.scr + (int64_t)blockIdx.x * a.scr_stride;
  double* X1 = w;                        // M n: X_1, then Q_1
  double* X3 = X1 + (int64_t)M * n;
  double* Xs = X3 + (int64_t)M * n;
  double* Qs = Xs + (int64_t)M * n;
  double* R1 = Qs + (int64_t)M * n;      // n x n
  double* R3 = R1 + n * n;
  double* M2 = R3 + n * n;               // [k4][k7][o2][s2]: D D D2 2
  double* Wt = M2 + 2 * (int64_t)D2 * D2;  // [a1][s1][k7][o2][s2]: 2n D D2 2 (<= 4 n D D2)
  double* Tb = Wt + 4 * (int64_t)n * D * D2;  // D x (2 n2 2 r3) (<= 4 n D D2)
  double* Ta = Tb + 4 * (int64_t)n * D * D2;  // (2 r1) x (2 n2 2 r3) (<= 8 n^2 D2)
  double* H1 = Ta + 8 * (int64_t)n * n * D2;  // (2n)^2
  double* H2 = H1 + 4 * n * n;
  double* U1 = H2 + 4 * n * n;           // 2n x D
  double* V3 = U1 + 2 * n * D;           // 2n x D (right singular vectors of the second split)
  double* Tc = V3 + 2 * n * D;           // (D 2 n2) x D
  double* ev = Tc + 2 * (int64_t)D2 * D2;  // 2 x 64
  double* refl = ev + 128;
  const double* lam4 = a.lam + (int64_t)link4 * D;
  const double* lam7 = a.lam + (int64_t)link7 * D;

  // (b) the end sites, QR-reduced
  const int r1 = su_reduce(a, S1, X1, R1, D, Xs, Qs);
  const int r3 = su_reduce(a, S3, X3, R3, D, Xs, Qs);
  // B_2 with its outer lambdas: M2[k4][k7][o2][s2]
  for (int e = tid; e < D * D * n2 * 2; e += WG) {
    const int s2 = e % 2, o = (e / 2) % n2, k7 = (e / (2 * n2)) % D, k4 = e / (2 * n2 * D);
    int idx[4];
    idx[l21] = k4; idx[l23] = k7;
    idx[o2[1]] = o % d2[o2[1]];
    idx[o2[0]] = o / d2[o2[1]];
    double lp = 1.0;
    for (int j = 0; j < 2; ++j)
      if (o2link[j] >= 0) lp *= a.lam[(int64_t)o2link[j] * D + idx[o2[j]]];
    const int off = ((idx[0] * d2[1] + idx[1]) * d2[2] + idx[2]) * d2[3] + idx[3];
    M2[e] = a.B[base2 + (int64_t)s2 * size2 + off] * lp;
  }
  __syncthreads();
  // (c) Wt[a1][s1][k7][o2][s2] = sum_k4 R1[a1][(s1,k4)] lambda_4 M2[k4][k7][o2][s2]
  const int nw = r1 * 2 * D * n2 * 2;
  for (int e = tid; e < nw; e += WG) {
    const int s2 = e % 2, o = (e / 2) % n2, k7 = (e / (2 * n2)) % D, s1 = (e / (2 * n2 * D)) % 2,
              a1 = e / (2 * n2 * D * 2);
    double acc = 0.0;
    for (int k4 = 0; k4 < D; ++k4)
      acc += R1[a1 * n + s1 * D + k4] * lam4[k4] * M2[((k4 * D + k7) * n2 + o) * 2 + s2];
    Wt[e] = acc;
  }
  __syncthreads();
  // T_a rows (a1, t1), columns (s2, o2, t3, a3), with the gate on (s1, s3)
  const double ga = exp(-0.25 * a.dt * a.J), gb = exp(0.75 * a.dt * a.J);
  const int R = 2 * r1, C = 2 * n2 * 2 * r3;
  for (int e = tid; e < r1 * 2 * n2 * r3; e += WG) {
    const int a3 = e % r3, o = (e / r3) % n2, s2 = (e / (r3 * n2)) % 2, a1 = e / (r3 * n2 * 2);
    double P[2][2];
    for (int s1 = 0; s1 < 2; ++s1)
      for (int s3 = 0; s3 < 2; ++s3) {
        double acc = 0.0;
        for (int k7 = 0; k7 < D; ++k7)
          acc += Wt[(((a1 * 2 + s1) * D + k7) * n2 + o) * 2 + s2] * lam7[k7] * R3[a3 * n + s3 * D + k7];
        P[s1][s3] = acc;
      }
    for (int t1 = 0; t1 < 2; ++t1)
      for (int t3 = 0; t3 < 2; ++t3) {
        double v = 0.0;
        for (int s1 = 0; s1 < 2; ++s1)
          for (int s3 = 0; s3 < 2; ++s3) v += su_gate(ga, gb, t1, t3, s1, s3) * P[s1][s3];
        Ta[(int64_t)(a1 * 2 + t1) * C + ((s2 * n2 + o) * 2 + t3) * r3 + a3] = v;
      }
  }
  __syncthreads();
  // (d) first split: U1, lambda~_4; Tb = lambda~_4 T_b = U1^T T_a / ||sigma||
  for (int e = tid; e < R * R; e += WG) {
    const int i = e / R, j = e % R;
    double acc = 0.0;
    for (int c = 0; c < C; ++c) acc += Ta[(int64_t)i * C + c] * Ta[(int64_t)j * C + c];
    H1[e] = acc;
  }
  __syncthreads();
  const int k01 = min(D, min(R, C));
  double inv1;
  const int kk1 = su_top(H1, R, k01, U1, ev, refl, lds, &s_kk, &inv1);
  for (int e = tid; e < D * C; e += WG) {
    const int i = e / C, c = e % C;
    double v = 0.0;
    if (i < kk1)
      for (int r = 0; r < R; ++r) v += U1[r * k01 + i] * Ta[(int64_t)r * C + c];
    Tb[e] = v * inv1;
  }
  __syncthreads();
  // (e) second split of Tb as rows (i4, s2, o2) x columns (t3, a3): V3, lambda~_7, T_c
  const int R2 = D * 2 * n2, C2 = 2 * r3;
  for (int e = tid; e < C2 * C2; e += WG) {
    const int i = e / C2, j = e % C2;
    double acc = 0.0;
    for (int r = 0; r < R2; ++r) acc += Tb[(int64_t)r * C2 + i] * Tb[(int64_t)r * C2 + j];
    H2[e] = acc;
  }
  __syncthreads();
  const int k02 = min(D, min(R2, C2));
  double inv2;
  const int kk2 = su_top(H2, C2, k02, V3, ev + 64, refl, lds, &s_kk, &inv2);
  for (int e = tid; e < R2 * D; e += WG) {
    const int r = e / D, i = e % D;
    double v = 0.0;
    if (i < kk2) {
      for (int c = 0; c < C2; ++c) v += Tb[(int64_t)r * C2 + c] * V3[c * k02 + i];
      v /= sqrt(fmax(ev[64 + i], 0.0));
    }
    Tc[e] = v;
  }
  __syncthreads();
  // (f) B_1 = Q_1 R~_1, (h) B_3 = Q_3 R~_3, outer lambdas divided out
  for (int e = tid; e < S1.m * n; e += WG) {
    const int o = e % S1.m, c = e / S1.m, t = c / D, i = c % D;
    double v = 0.0;
    if (i < kk1) {
      if (S1.m > n)
        for (int r = 0; r < r1; ++r) v += X1[o + (int64_t)r * S1.m] * U1[(r * 2 + t) * k01 + i];
      else
        v = U1[(o * 2 + t) * k01 + i];
    }
    double ip;
    const int off = su_addr(a, S1, o, i, &ip, true);
    a.B[S1.base + (int64_t)t * S1.size + off] = v * ip;
  }
  for (int e = tid; e < S3.m * n; e += WG) {
    const int o = e % S3.m, c = e / S3.m, t = c / D, i = c % D;
    double v = 0.0;
    if (i < kk2) {
      if (S3.m > n)
        for (int r = 0; r < r3; ++r) v += X3[o + (int64_t)r * S3.m] * V3[(t * r3 + r) * k02 + i];
      else
        v = V3[(t * r3 + o) * k02 + i];
    }
    double ip;
    const int off = su_addr(a, S3, o, i, &ip, true);
    a.B[S3.base + (int64_t)t * S3.size + off] = v * ip;
  }
  // (g) B_2 = T_c / lambda~_4 with its outer lambdas divided out
  for (int e = tid; e < D * 2 * n2 * D; e += WG) {
    const int i7 = e % D, o = (e / D) % n2, s2 = (e / (D * n2)) % 2, i4 = e / (D * n2 * 2);
    const double l4 = i4 < kk1 ? sqrt(fmax(ev[i4], 0.0)) * inv1 : 0.0;
    int idx[4];
    idx[l21] = i4; idx[l23] = i7;
    idx[o2[1]] = o % d2[o2[1]];
    idx[o2[0]] = o / d2[o2[1]];
    double ip = pinv(l4);
    for (int j = 0; j < 2; ++j)
      if (o2link[j] >= 0) ip *= pinv(a.lam[(int64_t)o2link[j] * D + idx[o2[j]]]);
    const int off = ((idx[0] * d2[1] + idx[1]) * d2[2] + idx[2]) * d2[3] + idx[3];
    a.B[base2 + (int64_t)s2 * size2 + off] = Tc[e] * ip;
  }
  __syncthreads();
  if (tid < D) {
    a.lam[(int64_t)link4 * D + tid] = tid < kk1 ? sqrt(fmax(ev[tid], 0.0)) * inv1 : 0.0;
    a.lam[(int64_t)link7 * D + tid] = tid < kk2 ? sqrt(fmax(ev[64 + tid], 0.0)) * inv2 : 0.0;
  }
}

// lambda <- 1 on every link entry.
__global__ void __launch_bounds__(WG) k_su_ones(double* lam, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) lam[i] = 1.0;
}

// out = mean over links of ||lam - prev|| / ||prev|| (one work-group, fixed order).
__global__ void __launch_bounds__(WG) k_su_mean(const double* lam, const double* prev, int n, int D, double* out) {
  double s = 0.0;
  for (int l = threadIdx.x; l < n; l += WG) {
    double dn = 0.0, on = 0.0;
    for (int i = 0; i < D; ++i) {
      const double o = prev[(int64_t)l * D + i], d = lam[(int64_t)l * D + i] - o;
      dn += d * d;
      on += o * o;
    }
    s += on > 0.0 ? sqrt(dn / on) : 0.0;
  }
  s = wg_sum(s);
  if (threadIdx.x == 0) *out = n > 0 ? s / n : 0.0;
}

// T = B with lambda^(1/2) contracted into both tensors of every link; one work-group per site.
__global__ void __launch_bounds__(WG) k_su_absorb(const double* B, const double* lam, const int64_t* offs,
                                                  const int32_t* dims, int Ly, int Lx, int D, double* T) {
  const int k = blockIdx.x, y = k / Lx, x = k % Lx;
  const int dl = dims[4 * k], du = dims[4 * k + 1], dr = dims[4 * k + 2], dd = dims[4 * k + 3];
  const int size = dl * du * dr * dd;
  const int nh = Ly * (Lx - 1);
  const int lk[4] = {x > 0 ? y * (Lx - 1) + x - 1 : -1, y > 0 ? nh + (y - 1) * Lx + x : -1,
                     x < Lx - 1 ? y * (Lx - 1) + x : -1, y < Ly - 1 ? nh + y * Lx + x : -1};
  for (int e = threadIdx.x; e < 2 * size; e += WG) {
    const int r = e % size;
    const int id = r % dd, ir = (r / dd) % dr, iu = (r / (dd * dr)) % du, il = r / (dd * dr * du);
    const int idx[4] = {il, iu, ir, id};
    double f = 1.0;
    for (int q = 0; q < 4; ++q)
      if (lk[q] >= 0) f *= sqrt(lam[(int64_t)lk[q] * D + idx[q]]);
    T[offs[k] + e] = B[offs[k] + e] * f;
  }
}

}  // namespace

int su_class_links(int Ly, int Lx, int cls) {
  if (cls == 0) return Ly * (Lx / 2);
  if (cls == 1) return Ly * ((Lx - 1) / 2);
  if (cls == 2) return (Ly / 2) * Lx;
  return ((Ly - 1) / 2) * Lx;
}

int64_t su_scratch_doubles(int D, bool nnn) {
  const int64_t n = 2 * D, M = (int64_t)D * D * D;
  const int64_t nn = 4 * M * n + 2 * n * n + 8 * n * n + 4 * n * D + 64 + EIG_PACK;
  return nnn ? std::max<int64_t>(nn, su_nnn_doubles(D)) : nn;
}

int su_class_plaquettes(int Ly, int Lx, int cls) { return ((Ly - (cls >> 1)) / 2) * ((Lx - (cls & 1)) / 2); }

void launch_su_init(double* lam, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_su_ones, dim3((unsigned)std::min<int64_t>((n + WG - 1) / WG, 1024)), dim3(WG), 0, s, lam, n);
}

void launch_su_class(double* B, double* lam, const int64_t* offs, const int32_t* dims, int Ly, int Lx, int D, int cls,
                     int first, int count, double dt, double J, double* scr, int64_t stride, hipStream_t s) {
  SuArgs a{B, lam, offs, dims, Ly, Lx, D, cls, first, dt, J, scr, stride, nullptr};
  hipLaunchKernelGGL(k_su_link, dim3(count), dim3(WG), 0, s, a);
}

void launch_su_nnn(double* B, double* lam, const int64_t* offs, const int32_t* dims, int Ly, int Lx, int D, int cls,
                   int anti, int first, int count, double dt, double J, double* scr, int64_t stride, hipStream_t s) {
  SuArgs a{B, lam, offs, dims, Ly, Lx, D, cls, first, dt, J, scr, stride, nullptr};
  hipLaunchKernelGGL(k_su_nnn, dim3(count), dim3(WG), 0, s, a, anti);
}

void launch_su_mean(const double* lam, const double* prev, int n, int D, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_su_mean, dim3(1), dim3(WG), 0, s, lam, prev, n, D, out);
}

void launch_su_absorb(const double* B, const double* lam, const int64_t* offs, const int32_t* dims, int Ly, int Lx,
                      int D, double* T, hipStream_t s) {
  hipLaunchKernelGGL(k_su_absorb, dim3(Ly * Lx), dim3(WG), 0, s, B, lam, offs, dims, Ly, Lx, D, T);
}

}  // namespace vp
