// Spin-inversion symmetrised amplitude (Sec. II.B, symmetrised wave function):
// Phi(S) = Psi(S) + Psi(Sbar), Sbar = S with every spin reversed.
//
// The evaluation of S and of Sbar each give (sign, log|Psi|, E_loc).  Since the
// Heisenberg elements are invariant under the reversal,
//   sum_S' <S|H|S'> Psi(Sbar') = sum_S' <Sbar|H|Sbar'> Psi(Sbar') = Psi(Sbar) E_loc(Sbar),
// so E_Phi(S) = (Psi(S) E_loc(S) + Psi(Sbar) E_loc(Sbar)) / (Psi(S) + Psi(Sbar)).
// The amplitudes enter relative to exp(max(log|Psi(S)|, log|Psi(Sbar)|)), so no
// exponential overflows.  w = |Phi(S)|^2 / |Psi(S)|^2 is the weight that turns a
// sample of |Psi|^2 into one of |Phi|^2; it is returned as log w.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vp_kernels.hpp"

namespace vp {

namespace {

constexpr int SIS_WG = 256;

__global__ void __launch_bounds__(SIS_WG) k_reverse_spins(const int8_t* __restrict__ s, int8_t* __restrict__ t,
                                                          int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)SIS_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * SIS_WG)
    t[i] = (int8_t)(1 - s[i]);
}

// In place over the outputs of S: (log|Psi|, sign, E_loc) -> (log|Phi|, sign, E_Phi).
__global__ void __launch_bounds__(SIS_WG) k_sis_combine(int n, double* __restrict__ log_abs, int8_t* __restrict__ sign,
                                                        double* __restrict__ e_loc, const double* __restrict__ log_abs_r,
                                                        const int8_t* __restrict__ sign_r,
                                                        const double* __restrict__ e_loc_r, double* __restrict__ log_w) {
  const int i = blockIdx.x * SIS_WG + threadIdx.x;
  if (i >= n) return;
  const double la = log_abs[i], lb = log_abs_r[i];
  const double m = fmax(la, lb);
  const double pa = (double)sign[i] * exp(la - m);
  const double pb = (double)sign_r[i] * exp(lb - m);
  const double phi = pa + pb;
  if (phi == 0.0) {  // Psi(Sbar) = -Psi(S): the configuration has no weight under |Phi|^2
    log_abs[i] = -INFINITY;
    sign[i] = 0;
    e_loc[i] = 0.0;
    log_w[i] = -INFINITY;
    return;
  }
  const double lphi = m + log(fabs(phi));
  e_loc[i] = (pa * e_loc[i] + pb * e_loc_r[i]) / phi;
  log_abs[i] = lphi;
  sign[i] = phi > 0.0 ? 1 : -1;
  log_w[i] = 2.0 * (lphi - la);
}

// Pair c of the |Phi|^2 chains: S at c, Sbar at c + h; outputs [h][n_meas], row m.
__global__ void __launch_bounds__(SIS_WG) k_pair_combine(int h, int n_meas, int m, const double* __restrict__ log_abs,
                                                         const int8_t* __restrict__ sign,
                                                         const double* __restrict__ e_loc, double* __restrict__ out_la,
                                                         int8_t* __restrict__ out_sg, double* __restrict__ out_e) {
  const int c = blockIdx.x * SIS_WG + threadIdx.x;
  if (c >= h) return;
  const int64_t o = (int64_t)c * n_meas + m;
  const double la = log_abs[c], lb = log_abs[c + h];
  const double mx = fmax(la, lb);
  const double pa = (double)sign[c] * exp(la - mx);
  const double pb = (double)sign[c + h] * exp(lb - mx);
  const double phi = pa + pb;
  if (phi == 0.0) {  // no weight under |Phi|^2 (only a start can be here)
    out_la[o] = -INFINITY;
    out_sg[o] = 0;
    out_e[o] = 0.0;
    return;
  }
  out_la[o] = mx + log(fabs(phi));
  out_sg[o] = phi > 0.0 ? 1 : -1;
  out_e[o] = (pa * e_loc[c] + pb * e_loc[c + h]) / phi;
}

__global__ void __launch_bounds__(SIS_WG) k_pair_spins(int h, int n_meas, int m, int N, const int8_t* __restrict__ spins,
                                                       int8_t* __restrict__ out) {
  const int64_t n = (int64_t)h * N;
  for (int64_t i = blockIdx.x * (int64_t)SIS_WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * SIS_WG) {
    const int64_t c = i / N, k = i - c * N;
    out[(c * n_meas + m) * N + k] = spins[i];
  }
}

}  // namespace

void launch_pair_combine(int h, int n_meas, int m, const double* log_abs, const int8_t* sign, const double* e_loc,
                         const int8_t* spins, int N, double* out_log_abs, int8_t* out_sign, double* out_e_loc,
                         int8_t* out_spins, hipStream_t st) {
  if (h <= 0) return;
  k_pair_combine<<<(h + SIS_WG - 1) / SIS_WG, SIS_WG, 0, st>>>(h, n_meas, m, log_abs, sign, e_loc, out_log_abs,
                                                               out_sign, out_e_loc);
  if (out_spins) {
    const int64_t blocks = ((int64_t)h * N + SIS_WG - 1) / SIS_WG;
    k_pair_spins<<<(unsigned)(blocks < 4096 ? blocks : 4096), SIS_WG, 0, st>>>(h, n_meas, m, N, spins, out_spins);
  }
}

void launch_reverse_spins(const int8_t* s, int8_t* t, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t blocks = (n + SIS_WG - 1) / SIS_WG;
  k_reverse_spins<<<(unsigned)(blocks < 4096 ? blocks : 4096), SIS_WG, 0, st>>>(s, t, n);
}

void launch_sis_combine(int n, double* log_abs, int8_t* sign, double* e_loc, const double* log_abs_r,
                        const int8_t* sign_r, const double* e_loc_r, double* log_w, hipStream_t st) {
  if (n <= 0) return;
  k_sis_combine<<<(n + SIS_WG - 1) / SIS_WG, SIS_WG, 0, st>>>(n, log_abs, sign, e_loc, log_abs_r, sign_r, e_loc_r,
                                                              log_w);
}

}  // namespace vp
