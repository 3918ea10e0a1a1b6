// Simple-update imaginary-time evolution (App. A), nearest-neighbour terms.
//
// The PEPS is held as site tensors B (the canonical flat layout of the
// parameters) and a diagonal matrix lambda on every link (D numbers per link:
// horizontal links (y,x)-(y,x+1) first, row-major, then vertical links
// (y,x)-(y+1,x)).  A step applies exp(-dt J S_A.S_B) once to every link, in
// four classes: horizontal links with x even, with x odd, vertical links with
// y even, with y odd.  Links of one class share no site, so one work-group per
// link updates a class in any order with the same result.  Per link (App. A,
// Fig. 7 (b)-(h), two sites):
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
// All of it in float64.
#include <hip/hip_runtime.h>

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
  double* change;       // [n_links] relative change of each link's lambda
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
  // the link's new lambda and its relative change (every thread has read the old one)
  __syncthreads();
  double dn = 0.0, on = 0.0;
  for (int i = 0; i < kd; ++i) {
    const double nv = i < kk ? sqrt(fmax(ev[i], 0.0)) * inv_nrm : 0.0;
    const double ov = lam_bond[i];
    dn += (nv - ov) * (nv - ov);
    on += ov * ov;
  }
  __syncthreads();
  if (tid < kd) a.lam[(int64_t)link * a.D + tid] = tid < kk ? sqrt(fmax(ev[tid], 0.0)) * inv_nrm : 0.0;
  if (tid == 0) a.change[link] = on > 0.0 ? sqrt(dn / on) : 0.0;
}

// lambda <- 1 on every link entry.
__global__ void __launch_bounds__(WG) k_su_ones(double* lam, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) lam[i] = 1.0;
}

// out = mean of change[0..n) (one work-group, fixed order).
__global__ void __launch_bounds__(WG) k_su_mean(const double* change, int n, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += WG) s += change[i];
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

int64_t su_scratch_doubles(int D) {
  const int64_t n = 2 * D, M = (int64_t)D * D * D;
  return 4 * M * n + 2 * n * n + 8 * n * n + 4 * n * D + 64 + EIG_PACK;
}

void launch_su_init(double* lam, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_su_ones, dim3((unsigned)std::min<int64_t>((n + WG - 1) / WG, 1024)), dim3(WG), 0, s, lam, n);
}

void launch_su_class(double* B, double* lam, const int64_t* offs, const int32_t* dims, int Ly, int Lx, int D, int cls,
                     int first, int count, double dt, double J, double* scr, double* change, hipStream_t s) {
  SuArgs a{B, lam, offs, dims, Ly, Lx, D, cls, first, dt, J, scr, su_scratch_doubles(D), change};
  hipLaunchKernelGGL(k_su_link, dim3(count), dim3(WG), 0, s, a);
}

void launch_su_mean(const double* change, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_su_mean, dim3(1), dim3(WG), 0, s, change, n, out);
}

void launch_su_absorb(const double* B, const double* lam, const int64_t* offs, const int32_t* dims, int Ly, int Lx,
                      int D, double* T, hipStream_t s) {
  hipLaunchKernelGGL(k_su_absorb, dim3(Ly * Lx), dim3(WG), 0, s, B, lam, offs, dims, Ly, Lx, D, T);
}

}  // namespace vp
