// Host-visible description of one lattice's device state and the phase-kernel
// launchers (implemented in vp_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vp {

// Per-chain scalar state kept on the device.
struct ChainMeta {
  int64_t sweep;        // Philox counter word 1 of the next sweep
  int64_t accepted;
  int64_t proposed;
  double e_acc;         // E_loc accumulator of the current measurement
  double logpsi;        // log|Psi| of the last top-down pass
  int32_t sign;         // sign of Psi
  int32_t flags;        // bit 0: zero amplitude, bit 1: non-finite value
  int64_t p_accepted;   // learned plaquette moves
  int64_t p_proposed;
};

enum : int32_t { FLAG_ZERO = 1, FLAG_NONFINITE = 2 };

// Everything a kernel needs to locate one chain's data.  Sizes are padded:
// every virtual leg has dimension d = D and every boundary bond c = Dc; true
// (smaller) dimensions are realised by zero entries.
struct LatDev {
  int Ly, Lx, d, c, N;
  double J1;
  double Jd, Ja;  // couplings of the diagonal (y,x)-(y+1,x+1) and the anti-diagonal (y,x+1)-(y+1,x)
  double Jk;      // coupling of the knight bonds (y,x)-(y+1,x+2) (triangular lattice), 0 otherwise
  int n_chains;
  uint64_t seed;
  int lat_id;
  // padded working tensors [N][2][d^4] (float or double), element type by kernel
  const void* Tw;
  // per-chain workspace (element type T), ints, doubles
  void* ws;
  int64_t ws_stride;
  int32_t* iws;
  int64_t iws_stride;
  double* dws;
  int64_t dws_stride;
  ChainMeta* meta;
  int8_t* spins;            // [n_chains][N]
  double* trace;            // [n_chains][n_bonds][2] (rho, accepted) of the last sweep, or null
  int n_bonds;              // Ly(Lx-1) + (Ly-1)Lx
  const void* net;          // proposal network parameters in the working precision, or null
  const void* net_bf;       // their packed bf16 copy (bf16 inference in the bf16 sampling mode)
  int learned;              // learned plaquette moves in the persistent sweep kernel
  int tile;                 // tile variant of the fused 2-row step (per-phase launches): 0, 1, 2
  int cmode;                // boundary truncation: 0 canonical SVD compression, 1 variational fit
  int fit_sweeps;           // sweeps of the variational fit
  const int32_t* kU;        // bond dims of U_y: kU[(y+1)*(Lx+1) + j], y = -1..Ly-1
  const int32_t* kD;        // bond dims of D_y: kD[y*(Lx+1) + j], y = 0..Ly
  const int32_t* dims;      // true leg dims per site [N][4] (l,u,r,d)
  const int64_t* coff;      // compact log-derivative offset per site [N+1]
  // workspace offsets (elements of T)
  int64_t oUb, oDb;         // boundaries: [(Ly+1)][Lx][c*d*c]
  int64_t oL3, oR3, oT3;    // 3-line envs: [(Lx+1)] slots each, 4 temps
  int64_t oL4, oR4, oT4;    // 4-line envs: [(Lx+1)] slots each, 4 temps
  int64_t oX0, oX1;         // GEMM intermediates [c*c*d*d*d]
  int64_t oDl;              // defect tensor scratch [d^4]
  // float64 compression workspace (per chain)
  double* cws;
  int64_t cws_stride;
  int64_t cG;               // Gram matrices [Lx][c*d*d*c]
  int64_t cX0, cX1;         // intermediates [c*c*d*d*d]
  int64_t cY, cW, cH, cHc, cVk;   // [c*c*d*d]
  int64_t cVp, cTa, cTb;    // [c*d*c]
  int64_t cRefl;            // Householder vectors [128*129/2]
  int64_t cLam;             // eigenvalues [64]
  // int offsets: exponents of env slots
  int64_t ieL3, ieR3, ieT3, ieL4, ieR4, ieT4;
  // double offsets
  int64_t dlamU, dlamD;     // [(Ly+1)] cumulative log-scales
};

// Outputs of one measured sweep (all may be null except where stated).
struct SampleOut {
  double* log_abs_psi;  // [chain][n_meas]
  int8_t* sign;
  double* e_loc;
  void* dlnpsi;         // [chain][n_meas][Np/2]
  int8_t* spins;        // [chain][n_meas][N]
  double* ratios;       // [chain][n_pairs] (vp_eval only)
  int n_meas;
  int m;                // index of this measurement (dyn_m == 0)
  int dyn_m;            // 1: the index is the chain's sweep counter minus sweep0
  int64_t sweep0;
  int64_t np_half;
  int n_pairs;
  int psi_meas;         // Psi from the measurement pass (bottom row) instead of the sampling pass
  double* plaq;         // [chain][(Ly-1)(Lx-1)] plaquette-flip ratios, or null
};

template <typename T> void launch_prepare_tensors(const LatDev& L, const double* Tflat, T* Tw,
                                                  const int64_t* offs, hipStream_t s);
template <typename T> void launch_init_trivial(const LatDev& L, hipStream_t s);
template <typename T> void launch_row3_right(const LatDev& L, int y, int ub_slot, int db_slot, bool bf16, hipStream_t s);
template <typename T> void launch_hsweep(const LatDev& L, int y, int last_row, bool bf16, hipStream_t s);
template <typename T> void launch_row4_right(const LatDev& L, int y, bool bf16, hipStream_t s);
template <typename T> void launch_vsweep(const LatDev& L, int y, bool bf16, bool learned, hipStream_t s);
// Chains of |Phi|^2: the decision phases over the pairs (ch, ch + n_chains/2), grid n_chains/2.
template <typename T> void launch_hsweep_pair(const LatDev& L, int y, int last_row, bool bf16, hipStream_t s);
template <typename T> void launch_vsweep_pair(const LatDev& L, int y, bool bf16, hipStream_t s);
// Persistent whole-sweep launch over (lattice, chain) items; lats/outs/items/next are device arrays,
// L0 a host copy of any of the lattices (they share d, c and the working type).
template <typename T> void launch_sweep_queue(const LatDev& L0, const LatDev* lats, const SampleOut* outs,
                                              int measure, const int2* items, int n_items, int* next, bool bf16,
                                              int grid, hipStream_t s);
template <typename T> int sweep_queue_occupancy(const LatDev& L0, bool bf16);
template <typename T> void launch_compress(const LatDev& L, int y, int upper, hipStream_t s);
template <typename T> void launch_measure3(const LatDev& L, int y, const SampleOut& o, hipStream_t s);
template <typename T> void launch_measure4(const LatDev& L, int y, const SampleOut& o, hipStream_t s);
template <typename T> void launch_psi_fixed(const LatDev& L, hipStream_t s);
void launch_begin_sample(const LatDev& L, hipStream_t s);
void launch_finish_sample(const LatDev& L, const SampleOut& o, int n_active, hipStream_t s);
void launch_next_sweep(const LatDev& L, hipStream_t s);
void launch_init_tensors(double* T, int64_t Np, uint64_t seed, int lat_id, double scale, double perturb,
                         hipStream_t s);
void launch_init_chains(const LatDev& L, hipStream_t s);
void launch_copy_spins(const LatDev& L, const int8_t* src, int n_cfg, hipStream_t s);
template <typename T> void launch_gradient(const int64_t* offs, const int64_t* coff, const int32_t* sz,
                                           int N, int64_t Np, const double* e, const T* dl,
                                           const int8_t* spins, int64_t ns, double* grad, double* emean,
                                           double* work, hipStream_t s);
template <typename T>
int launch_sr(const int64_t* offs, const int64_t* coff, const int32_t* sz, int N, int64_t np, const double* e,
              const T* dl, const int8_t* spins, int64_t ns, double shift, double lr, double* Tm,
              double* delta_out, double* work, int* flag, hipStream_t s);
int64_t sr_work_doubles(int64_t np, int64_t ns);
void launch_sign_sgd(double* T, const double* g, int64_t Np, double step_len, uint64_t seed, int lat_id,
                     uint64_t step, hipStream_t s);

// Proposal network (batched, float32): work holds net_work_floats(n, H, W)
// floats; part [n] doubles, cnt [n] ints, scal [2] doubles.
size_t net_work_floats(int n, int H, int W);
// Floats net_forward uses of its work buffer (a prefix of net_work_floats).
size_t net_forward_floats(int n, int H, int W);
// The static forward-pass scratch: NET_SCRATCH_FLOATS floats per GPU.
// net_scratch_setup looks up the calling process's copy on `device` once (with
// that device current); net_scratch_ptr returns it, or null before the setup.
constexpr size_t NET_SCRATCH_FLOATS = size_t(4) << 20;  // 16 MiB
hipError_t net_scratch_setup(int device);
float* net_scratch_ptr(int device);
void net_forward(const float* th, const int8_t* spins, int n, int H, int W, float* work, float* logits,
                 hipStream_t s);
void net_loss_grad(const float* th, const int8_t* spins, const double* ratios, int n, int H, int W, float* work,
                   double* part, int* cnt, double* scal, float* grad, hipStream_t s);
void net_adam(float* th, const float* g, float* m, float* v, float lr, int t, hipStream_t s);
void net_gather(const int8_t* spins, const double* ratios, const int32_t* idx, int nb, int H, int W, int8_t* sb,
                double* rb, hipStream_t s);
void net_cast_f64(const float* src, double* dst, hipStream_t s);
// The packed bf16 copy of the parameters (NET_BF_BYTES bytes) for bf16 inference.
void net_pack_bf16(const float* src, void* dst, hipStream_t s);
// Logits of every plaquette of n configurations [n][(H-1)(W-1)] float64, as the
// learned sweep evaluates them: kind 0 float32 weights, 1 float64, 2 bf16 inference.
void net_local_logits(int kind, const float* w32, const double* w64, const void* wbf, const int8_t* spins, int n,
                      int H, int Wd, int flip, double* out, hipStream_t s);

// Simple update (vp_su.hip): links per class (0: horizontal x even, 1: x odd,
// 2: vertical y even, 3: y odd), plaquettes per class (y mod 2, x mod 2) =
// (cls >> 1, cls & 1), per-work-group scratch (doubles; nnn: large enough for
// the three-site update too), lambda <- 1, one launch over links (or
// plaquettes' diagonals) first .. first+count-1 of a class, the mean relative
// change of the lambdas against those at the start of the step, and the
// absorption of lambda^(1/2) into T.
int su_class_links(int Ly, int Lx, int cls);
int su_class_plaquettes(int Ly, int Lx, int cls);
int64_t su_scratch_doubles(int D, bool nnn);
void launch_su_init(double* lam, int64_t n, hipStream_t s);
void launch_su_class(double* B, double* lam, const int64_t* offs, const int32_t* dims, int Ly, int Lx, int D, int cls,
                     int first, int count, double dt, double J, double* scr, int64_t stride, hipStream_t s);
void launch_su_nnn(double* B, double* lam, const int64_t* offs, const int32_t* dims, int Ly, int Lx, int D, int cls,
                   int anti, int first, int count, double dt, double J, double* scr, int64_t stride, hipStream_t s);
void launch_su_mean(const double* lam, const double* prev, int n, int D, double* out, hipStream_t s);
void launch_su_absorb(const double* B, const double* lam, const int64_t* offs, const int32_t* dims, int Ly, int Lx,
                      int D, double* T, hipStream_t s);

// Spin-inversion symmetrisation: t = reversed s (n bytes); the outputs of S
// combined in place with those of Sbar into log|Phi|, sign, E_Phi and log w.
void launch_reverse_spins(const int8_t* s, int8_t* t, int64_t n, hipStream_t st);
void launch_sis_combine(int n, double* log_abs, int8_t* sign, double* e_loc, const double* log_abs_r,
                        const int8_t* sign_r, const double* e_loc_r, double* log_w, hipStream_t st);
// The pair sampler's measurement: pair c's S values at index c and Sbar values
// at c + h of (log_abs, sign, e_loc) combined into row m of the [h][n_meas]
// outputs, and the S configuration (spins [2h][N]) into spins_out (may be null).
void launch_pair_combine(int h, int n_meas, int m, const double* log_abs, const int8_t* sign, const double* e_loc,
                         const int8_t* spins, int N, double* out_log_abs, int8_t* out_sign, double* out_e_loc,
                         int8_t* out_spins, hipStream_t st);

// Column-wise vertical bonds (vp_cols.hip): the transposed lattice's tensors
// (T' from T: offs / offs_t the two lattices' site offsets, dims the row
// lattice's leg dimensions) and configurations ([n_chains][N], to or from the
// transposed site order), its horizontal ratios placed as the row lattice's
// vertical ones (rt [n][npt] -> r [n][np]), its energies added into row m of
// the [n][n_meas] outputs, and its move counts added to (accepted, proposed)
// at the start of every stride-long row of out [n][stride].
void launch_transpose_tensors(const double* T, double* Tt, const int64_t* offs, const int64_t* offs_t,
                              const int32_t* dims, int Ly, int Lx, hipStream_t s);
void launch_transpose_spins(const int8_t* src, int8_t* dst, int n_chains, int Ly, int Lx, bool to_columns,
                            hipStream_t s);
void launch_column_ratios(const double* rt, int npt, double* r, int np, int n, int Ly, int Lx, hipStream_t s);
void launch_add_energy(double* e, int n_meas, int m, const double* et, int n, hipStream_t s);
// The triangular lattice's knight bonds (y,x)-(y+2,x+1) (row-major from base_r of r
// [n][np]) from the transposed lattice's (x,y)-(x+1,y+2) bonds (from base_t of rt [n][npt]).
void launch_knight_ratios(const double* rt, int npt, int base_t, double* r, int np, int base_r, int n, int Ly, int Lx,
                          hipStream_t s);
void launch_add_counts(const ChainMeta* b, int64_t* out, int stride, int n, hipStream_t s);

}  // namespace vp
