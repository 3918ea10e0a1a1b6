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

}  // namespace

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
