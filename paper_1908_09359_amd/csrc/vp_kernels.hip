// Phase kernels of the VMC-PEPS hot path.  Each launch covers every chain of a
// lattice (grid = chains, one 256-thread work-group per chain) and performs one
// phase of a sweep for one row: right environments, the horizontal or vertical
// Metropolis pass, the boundary compression, or the measurement of a row.
#include "vp_device.hpp"
#include "vp_eig.hpp"
#include "vp_env4.hpp"
#include "vp_env4bf.hpp"
#include "vp_env3.hpp"
#include "vp_fit.hpp"
#include "vp_kernels.hpp"
#include "vp_net.hpp"

#include <math.h>

#include <type_traits>

#ifndef VP_KERNEL_UNIT
#define VP_KERNEL_UNIT 0
#endif

namespace vp {

namespace {

template <typename T>
struct Chain {
  T* ws;
  int32_t* iw;
  double* dw;
  ChainMeta* meta;
  int8_t* sp;
  int id;  // chain index within its lattice (Philox counter word 0, output row)
};

template <typename T>
__device__ inline Chain<T> chain_of(const LatDev& L, int ch) {
  Chain<T> C;
  C.ws = (T*)L.ws + (int64_t)ch * L.ws_stride;
  C.iw = L.iws + (int64_t)ch * L.iws_stride;
  C.dw = L.dws + (int64_t)ch * L.dws_stride;
  C.meta = L.meta + ch;
  C.sp = L.spins + (int64_t)ch * L.N;
  C.id = ch;
  return C;
}

__device__ inline S4 st_std(int d) { return S4{d * d * d, d * d, d, 1}; }
__device__ inline S4 st_mirror(S4 s) { return S4{s.r, s.u, s.l, s.d}; }
__device__ inline S4 st_swapud(S4 s) { return S4{s.l, s.d, s.r, s.u}; }
__device__ inline S3 sb_std(int c, int d) { return S3{d * c, c, 1}; }
__device__ inline S3 sb_mirror(int c, int d) { return S3{1, c, d * c}; }

template <typename T>
__device__ inline const T* tw(const LatDev& L, int k, int s) {
  const int d4 = L.d * L.d * L.d * L.d;
  return (const T*)L.Tw + ((int64_t)k * 2 + s) * d4;
}

// Boundary site: slot holds U_{slot-1} (upper) or D_slot (lower).
template <typename T>
__device__ inline T* ub(const LatDev& L, const Chain<T>& C, int slot, int x) {
  return C.ws + L.oUb + ((int64_t)slot * L.Lx + x) * (L.c * L.d * L.c);
}
template <typename T>
__device__ inline T* db(const LatDev& L, const Chain<T>& C, int slot, int x) {
  return C.ws + L.oDb + ((int64_t)slot * L.Lx + x) * (L.c * L.d * L.c);
}

__device__ inline int e3sz(const LatDev& L) { return L.c * L.d * L.c; }
__device__ inline int e4sz(const LatDev& L) { return L.c * L.d * L.d * L.c; }

template <typename T>
__device__ inline void set_unit(T* x_p, int n) {
  auto* x = gmem(x_p);
  for (int i = threadIdx.x; i < n; i += WG) x[i] = (i == 0) ? T(1) : T(0);
  __syncthreads();
}

__device__ inline void raise_flag(ChainMeta* m, int f) {
  if (threadIdx.x == 0) atomicOr(&m->flags, f);
}

// Whether a chain has an error flag, decided once for the whole work-group
// (a kernel on another stream may raise a flag of the same chain meanwhile).
__device__ inline bool chain_flagged(const ChainMeta* m) {
  __shared__ int f;
  if (threadIdx.x == 0) f = m->flags;
  __syncthreads();
  const bool v = f != 0;
  __syncthreads();
  return v;
}

// Row of this measurement in the outputs: fixed, or from the sweep counter
// (so that one captured sweep serves every measured sweep of a call).
__device__ inline int64_t meas_index(const SampleOut& o, const ChainMeta* m) {
  return o.dyn_m ? m->sweep - o.sweep0 : (int64_t)o.m;
}

// 3-line column step with optional flipped site: t = T[s ^ flip].  (DD, CC)
// with DD*DD = 64 and DD*CC = 128 select the fused MFMA step in the working
// precision, also for a bf16 sampling pass (it is faster there than the
// generic bf16-operand step); otherwise the generic strided-GEMM step runs.
template <typename T, int DD, int CC>
constexpr bool fused3() {
  if constexpr (DD > 0) return Env3Shape<DD, CC>::ok;
  else return false;
}
template <typename T, int DD, int CC, bool BF16 = false>
__device__ inline int step3(const LatDev& L, const Chain<T>& C, T* out, const T* in, int y, int x,
                            int flip, const T* Ux, const T* Dx, bool right, lds_char* tiles_l) {
  char* tiles = (char*)tiles_l;
  int k = y * L.Lx + x;
  const T* t = tw<T>(L, k, C.sp[k] ^ flip);
  S4 st = st_std(L.d);
  if constexpr (fused3<T, DD, CC>()) {
    if (right)
      env3_fused<T, DD, CC>(out, in, Ux, sb_mirror(CC, DD), t, st_mirror(st), Dx, sb_mirror(CC, DD), tiles);
    else
      env3_fused<T, DD, CC>(out, in, Ux, sb_std(CC, DD), t, st, Dx, sb_std(CC, DD), tiles);
    return wg_renorm<T>(out, CC * DD * CC);
  }
  if (right)
    env3_step<T, BF16>(out, in, Ux, sb_mirror(L.c, L.d), t, st_mirror(st), Dx, sb_mirror(L.c, L.d),
                       C.ws + L.oX0, C.ws + L.oX1, L.c, L.d, tiles);
  else
    env3_step<T, BF16>(out, in, Ux, sb_std(L.c, L.d), t, st, Dx, sb_std(L.c, L.d), C.ws + L.oX0,
                       C.ws + L.oX1, L.c, L.d, tiles);
  return wg_renorm<T>(out, e3sz(L));
}

// LDS bytes of a kernel's 3-line column steps (and, with defects, its defect tensors).
template <typename T, int DD, int CC, bool BF16, bool DEFECT = false>
constexpr size_t step3_lds() {
  if constexpr (DD > 0) {
    if constexpr (Env3Shape<DD, CC>::ok) {
      constexpr size_t a = Env3Shape<DD, CC>::template lds_bytes<T>();
      constexpr size_t b = DEFECT ? Env3Shape<DD, CC>::template defect_lds_bytes<T>() : 0;
      return a > b ? a : b;
    }
  }
  return GEMM_TILE_BYTES;
}

// LDS bytes a kernel provides for its 2-row column steps.
template <typename TC, typename TB, int DD, int CC, bool GRAM = false, int BBX = 0>
constexpr size_t env4_lds() {
  if constexpr (DD > 0)
    return Env4Shape<DD, CC, (BBX > 0 ? BBX : env4_bb<TC, TB, DD, CC, GRAM>())>::template lds_bytes<TC, TB, GRAM>();
  else return GEMM_TILE_BYTES;  // the generic step's GEMM tiles
}

// 4-line column step over rows y and y+1; flip1/flip2 select the flipped slot.
// DD > 0 selects the fused MFMA step (environment layout [c][a][l1][l2]);
// DD == 0 the generic strided-GEMM step (layout [a][l1][l2][c]).  BF16: bf16
// operands with f32 accumulation.
template <typename T, int DD, int CC, bool BF16 = false, int BBX = 0>
__device__ inline int step4(const LatDev& L, const Chain<T>& C, T* out, const T* in, int y, int x,
                            int flip1, int flip2, const T* Ux, const T* Dx, bool right, lds_char* lds_l) {
  char* lds = (char*)lds_l;
  int k1 = y * L.Lx + x, k2 = (y + 1) * L.Lx + x;
  const T* t1 = tw<T>(L, k1, C.sp[k1] ^ flip1);
  const T* t2 = tw<T>(L, k2, C.sp[k2] ^ flip2);
  S4 st = st_std(L.d);
  const S3 sb = right ? sb_mirror(L.c, L.d) : sb_std(L.c, L.d);
  const S4 s = right ? st_mirror(st) : st;
  if constexpr (DD > 0 && BF16) {
    env4_bf16<DD, CC, T>(out, in, Ux, sb, t1, s, t2, s, Dx, sb, lds);
  } else if constexpr (DD > 0) {
    env4_fused<T, T, DD, CC, false, false, BBX>(out, in, Ux, sb, t1, s, t2, s, Dx, sb, lds);
  } else {
    env4_step<T, T, BF16>(out, in, Ux, sb, t1, s, t2, s, Dx, sb, C.ws + L.oX0, C.ws + L.oX1, L.c, L.d, lds);
  }
  return wg_renorm<T>(out, e4sz(L));
}

// value * 2^e as a double (exact scaling)
__device__ inline double scaled(double v, int e) { return ldexp(v, e); }

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(WG) k_prepare_tensors(LatDev L, const double* __restrict__ Tflat,
                                                        T* __restrict__ Tw, const int64_t* __restrict__ offs) {
  const int d = L.d, d4 = d * d * d * d;
  int64_t total = (int64_t)L.N * 2 * d4;
  for (int64_t i = blockIdx.x * (int64_t)WG + threadIdx.x; i < total; i += (int64_t)gridDim.x * WG) {
    int64_t k = i / (2 * d4);
    int rem = (int)(i - k * 2 * d4);
    int s = rem / d4, e = rem - s * d4;
    int l = e / (d * d * d), u = (e / (d * d)) % d, r = (e / d) % d, dd = e % d;
    int dl = L.dims[4 * k], du = L.dims[4 * k + 1], dr = L.dims[4 * k + 2], ddd = L.dims[4 * k + 3];
    T v = T(0);
    if (l < dl && u < du && r < dr && dd < ddd) {
      int64_t n = (int64_t)dl * du * dr * ddd;
      v = (T)Tflat[offs[k] + s * n + ((l * du + u) * dr + r) * ddd + dd];
    }
    Tw[i] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(WG) k_init_trivial(LatDev L) {
  Chain<T> C = chain_of<T>(L, blockIdx.x);
  const int sz = L.c * L.d * L.c;
  for (int x = 0; x < L.Lx; ++x) {
    set_unit<T>(ub<T>(L, C, 0, x), sz);
    set_unit<T>(db<T>(L, C, L.Ly, x), sz);
  }
  if (threadIdx.x == 0) {
    C.dw[L.dlamU + 0] = 0.0;
    C.dw[L.dlamD + L.Ly] = 0.0;
  }
}

// R3[x] = R(x) for x = Lx-1 .. 1 of the network <D|row y|U>; R3[Lx] = ones.
template <typename T, int DD, int CC, bool BF16>
__device__ __forceinline__ void ph_row3_right(const LatDev& L, int ch, int y, int ub_slot, int db_slot, char* tiles) {
  Chain<T> C = chain_of<T>(L, ch);
  const int sz = e3sz(L);
  T* R = C.ws + L.oR3;
  int* eR = C.iw + L.ieR3;
  set_unit<T>(R + (int64_t)L.Lx * sz, sz);
  if (threadIdx.x == 0) eR[L.Lx] = 0;
  for (int x = L.Lx - 1; x >= 1; --x) {
    int e = step3<T, DD, CC, BF16>(L, C, R + (int64_t)x * sz, R + (int64_t)(x + 1) * sz, y, x, 0,
                           ub<T>(L, C, ub_slot, x), db<T>(L, C, db_slot, x), true, as_lds(tiles));
    if (threadIdx.x == 0) eR[x] = eR[x + 1] + e;
    __syncthreads();
  }
}

__device__ inline bool metropolis(const LatDev& L, int ch, ChainMeta* meta, double num, double den, int esum,
                                  int bond) {
  if (den == 0.0) {
    raise_flag(meta, FLAG_ZERO);
    return false;
  }
  double rho = scaled(num / den, esum);
  double R = rho * rho;
  if (!isfinite(R)) {
    raise_flag(meta, FLAG_NONFINITE);
    return false;
  }
  U64x4 w = philox4x64_10((uint64_t)ch, (uint64_t)meta->sweep, (uint64_t)bond, TAG_METRO,
                          L.seed, (uint64_t)L.lat_id);
  double u = uniform53(w.v[0]);
  const bool acc = u < R;
  if (L.trace && threadIdx.x == 0) {
    double* t = L.trace + 2 * ((int64_t)ch * L.n_bonds + bond);
    t[0] = rho;
    t[1] = acc ? 1.0 : 0.0;
  }
  return acc;
}

// Trace entry of a bond whose pair is parallel (no move proposed).
__device__ inline void trace_skip(const LatDev& L, int ch, int bond) {
  if (L.trace && threadIdx.x == 0) {
    double* t = L.trace + 2 * ((int64_t)ch * L.n_bonds + bond);
    t[0] = 0.0;
    t[1] = 0.0;
  }
}

// Horizontal bonds of row y, left to right (Sec. II.A Eq. (9)).  With moves = 0
// no move is attempted.  For the last row the full amplitude is produced.
template <typename T, int DD, int CC, bool BF16>
__device__ __forceinline__ void ph_hsweep(const LatDev& L, int ch, int y, int last_row, int moves, char* tiles) {
  Chain<T> C = chain_of<T>(L, ch);
  if (chain_flagged(C.meta)) return;
  const int sz = e3sz(L);
  T* tmp = C.ws + L.oT3;
  const T* R = C.ws + L.oR3;
  const int* eR = C.iw + L.ieR3;
  int slot[4] = {0, 1, 2, 3};  // cur, nxt, f1, f2
  set_unit<T>(tmp + slot[0] * sz, sz);
  int ecur = 0;
  for (int x = 0; x < L.Lx - 1; ++x) {
    const T* Ux = ub<T>(L, C, y, x);
    const T* Dx = db<T>(L, C, y + 1, x);
    T* cur = tmp + slot[0] * sz;
    T* nxt = tmp + slot[1] * sz;
    int enxt = ecur + step3<T, DD, CC, BF16>(L, C, nxt, cur, y, x, 0, Ux, Dx, false, as_lds(tiles));
    const int k = y * L.Lx + x;
    bool acc = false;
    if (moves && C.sp[k] == C.sp[k + 1]) trace_skip(L, C.id, y * (2 * L.Lx - 1) + x);
    if (moves && C.sp[k] != C.sp[k + 1]) {
      T* f1 = tmp + slot[2] * sz;
      T* f2 = tmp + slot[3] * sz;
      int ef1 = ecur + step3<T, DD, CC, BF16>(L, C, f1, cur, y, x, 1, Ux, Dx, false, as_lds(tiles));
      int ef2 = ef1 + step3<T, DD, CC, BF16>(L, C, f2, f1, y, x + 1, 1, ub<T>(L, C, y, x + 1),
                                     db<T>(L, C, y + 1, x + 1), false, as_lds(tiles));
      double num = wg_dot<T>(f2, R + (int64_t)(x + 2) * sz, sz);
      double den = wg_dot<T>(nxt, R + (int64_t)(x + 1) * sz, sz);
      int bond = y * (2 * L.Lx - 1) + x;
      acc = metropolis(L, C.id, C.meta, num, den, ef2 + eR[x + 2] - enxt - eR[x + 1], bond);
      if (threadIdx.x == 0) {
        C.meta->proposed += 1;
        if (acc) {
          int8_t a = C.sp[k];
          C.sp[k] = C.sp[k + 1];
          C.sp[k + 1] = a;
          C.meta->accepted += 1;
        }
      }
      __syncthreads();
      if (acc) {  // column x now carries the exchanged tensor: f1 becomes current
        int t = slot[1]; slot[1] = slot[2]; slot[2] = t;
        enxt = ef1;
      }
    }
    int t = slot[0]; slot[0] = slot[1]; slot[1] = t;
    ecur = enxt;
  }
  if (last_row) {
    const int x = L.Lx - 1;
    T* cur = tmp + slot[0] * sz;
    T* nxt = tmp + slot[1] * sz;
    int e = ecur + step3<T, DD, CC, BF16>(L, C, nxt, cur, y, x, 0, ub<T>(L, C, y, x), db<T>(L, C, y + 1, x), false,
                                  as_lds(tiles));
    double v = (double)nxt[0];
    if (threadIdx.x == 0) {
      if (v == 0.0) {
        atomicOr(&C.meta->flags, FLAG_ZERO);
      } else if (!isfinite(v)) {
        atomicOr(&C.meta->flags, FLAG_NONFINITE);
      } else {
        C.meta->logpsi = C.dw[L.dlamU + y] + log(fabs(v)) + e * 0.69314718055994530942;
        C.meta->sign = v > 0 ? 1 : -1;
      }
    }
  }
}

// R4[x] for x = Lx-1 .. 1 of <D_{y+2}|M_{y+1} M_y|U_{y-1}>.
template <typename T, int DD, int CC, bool BF16, int BBX = 0>
__device__ __forceinline__ void ph_row4_right(const LatDev& L, int ch, int y, char* lds) {
  Chain<T> C = chain_of<T>(L, ch);
  if (chain_flagged(C.meta)) return;
  const int sz = e4sz(L);
  T* R = C.ws + L.oR4;
  int* eR = C.iw + L.ieR4;
  set_unit<T>(R + (int64_t)L.Lx * sz, sz);
  if (threadIdx.x == 0) eR[L.Lx] = 0;
  for (int x = L.Lx - 1; x >= 1; --x) {
    int e = step4<T, DD, CC, BF16, BBX>(L, C, R + (int64_t)x * sz, R + (int64_t)(x + 1) * sz, y, x, 0, 0,
                                   ub<T>(L, C, y, x), db<T>(L, C, y + 2, x), true, as_lds(lds));
    if (threadIdx.x == 0) eR[x] = eR[x + 1] + e;
    __syncthreads();
  }
}

// Vertical bonds between rows y and y+1, left to right.
// Propose-or-stay Metropolis-Hastings decision of a learned plaquette move:
// accept iff u < R pi(S')/pi(S), R = rho^2.
__device__ inline bool plaquette_accept(ChainMeta* meta, double num, double den, int esum, double pi_fwd,
                                        double pi_back, double u) {
  if (den == 0.0) {
    raise_flag(meta, FLAG_ZERO);
    return false;
  }
  const double rho = scaled(num / den, esum);
  const double R = rho * rho;
  if (!isfinite(R)) {
    raise_flag(meta, FLAG_NONFINITE);
    return false;
  }
  return u < R * pi_back / pi_fwd;
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

// Vertical bonds between rows y and y+1, left to right.  LEARN: after the
// vertical bond at x < Lx-1, the learned move of plaquette (y, x): proposed
// with probability pi = sigmoid(f_x(S)) (word 0 of Philox counter (chain,
// sweep, y(Lx-1)+x, 6)), accepted with min[1, R pi(S')/pi(S)] (word 1); R from
// the two-row network with columns x and x+1 exchanged in both rows.
template <typename T, int DD, int CC, bool BF16, bool LEARN, int BBX = 0>
__device__ __forceinline__ void ph_vsweep(const LatDev& L, int ch, int y, char* lds) {
  Chain<T> C = chain_of<T>(L, ch);
  if (chain_flagged(C.meta)) return;
  const int sz = e4sz(L);
  T* tmp = C.ws + L.oT4;
  const T* R = C.ws + L.oR4;
  const int* eR = C.iw + L.ieR4;
  int slot[4] = {0, 1, 2, 3};  // cur, nxt, f (and a fourth temp for plaquette moves)
  set_unit<T>(tmp + slot[0] * sz, sz);
  int ecur = 0;
  // a learned move at (y, x-1) has already contracted the network through
  // column x for the spins it left: that is this column's nxt (exponent epre)
  bool have_nxt = false;
  int epre = 0;
  for (int x = 0; x < L.Lx; ++x) {
    const T* Ux = ub<T>(L, C, y, x);
    const T* Dx = db<T>(L, C, y + 2, x);
    T* cur = tmp + slot[0] * sz;
    T* nxt = tmp + slot[1] * sz;
    const int vb = y * (2 * L.Lx - 1) + (L.Lx - 1) + x;
    if (C.sp[y * L.Lx + x] == C.sp[(y + 1) * L.Lx + x]) trace_skip(L, C.id, vb);
    if (x == L.Lx - 1 && !(C.sp[y * L.Lx + x] != C.sp[(y + 1) * L.Lx + x])) break;
    int enxt = have_nxt ? epre : ecur + step4<T, DD, CC, BF16, BBX>(L, C, nxt, cur, y, x, 0, 0, Ux, Dx, false,
                                                                       as_lds(lds));
    have_nxt = false;
    const int k1 = y * L.Lx + x, k2 = (y + 1) * L.Lx + x;
    if (C.sp[k1] != C.sp[k2]) {
      T* f = tmp + slot[2] * sz;
      int ef = ecur + step4<T, DD, CC, BF16, BBX>(L, C, f, cur, y, x, 1, 1, Ux, Dx, false, as_lds(lds));
      double num = wg_dot<T>(f, R + (int64_t)(x + 1) * sz, sz);
      double den = wg_dot<T>(nxt, R + (int64_t)(x + 1) * sz, sz);
      bool acc = metropolis(L, C.id, C.meta, num, den, ef - enxt, vb);
      if (threadIdx.x == 0) {
        C.meta->proposed += 1;
        if (acc) {
          int8_t a = C.sp[k1];
          C.sp[k1] = C.sp[k2];
          C.sp[k2] = a;
          C.meta->accepted += 1;
        }
      }
      __syncthreads();
      if (acc) {
        int t = slot[1]; slot[1] = slot[2]; slot[2] = t;
        enxt = ef;
      }
    }
    if constexpr (LEARN) {
      const int k1 = y * L.Lx + x, k2 = k1 + L.Lx;
      if (x < L.Lx - 1 && C.sp[k1] + C.sp[k1 + 1] + C.sp[k2] + C.sp[k2 + 1] == 2) {
        const int q = y * (L.Lx - 1) + x;
        U64x4 w = philox4x64_10((uint64_t)C.id, (uint64_t)C.meta->sweep, (uint64_t)q, TAG_PLAQ, L.seed,
                                (uint64_t)L.lat_id);
        // bf16 inference with the bf16 sampling steps, the working precision otherwise
        auto logit = [&](int flip) -> double {
          if constexpr (BF16) return net_logit_bf16(static_cast<const char*>(L.net_bf), C.sp, L.Ly, L.Lx, y, x, flip, lds);
          else return net_logit<T>(static_cast<const T*>(L.net), C.sp, L.Ly, L.Lx, y, x, flip, lds);
        };
        const double pi_fwd = net_sigmoid(logit(0));
        if (uniform53(w.v[0]) < pi_fwd) {
          const T* Ux1 = ub<T>(L, C, y, x + 1);
          const T* Dx1 = db<T>(L, C, y + 2, x + 1);
          T* cur = tmp + slot[0] * sz;
          T* nxt = tmp + slot[1] * sz;
          T* f1 = tmp + slot[2] * sz;
          T* f2 = tmp + slot[3] * sz;
          const int ef1 = ecur + step4<T, DD, CC, BF16, BBX>(L, C, f1, cur, y, x, 1, 1, Ux, Dx, false, as_lds(lds));
          const int ef2 = ef1 + step4<T, DD, CC, BF16, BBX>(L, C, f2, f1, y, x + 1, 1, 1, Ux1, Dx1, false, as_lds(lds));
          // the current network through column x+1, into the slot of cur (no longer needed)
          const int eden = enxt + step4<T, DD, CC, BF16, BBX>(L, C, cur, nxt, y, x + 1, 0, 0, Ux1, Dx1, false, as_lds(lds));
          const double num = wg_dot<T>(f2, R + (int64_t)(x + 2) * sz, sz);
          const double den = wg_dot<T>(cur, R + (int64_t)(x + 2) * sz, sz);
          const double pi_back = net_sigmoid(logit(1));
          const bool acc = plaquette_accept(C.meta, num, den, ef2 - eden, pi_fwd, pi_back, uniform53(w.v[1]));
          if (threadIdx.x == 0) {
            C.meta->p_proposed += 1;
            if (acc) {
              C.sp[k1] ^= 1; C.sp[k1 + 1] ^= 1; C.sp[k2] ^= 1; C.sp[k2 + 1] ^= 1;
              C.meta->p_accepted += 1;
            }
          }
          __syncthreads();
          if (acc) {  // column x now carries the flipped tensors: f1 is the environment through x
            int t = slot[1]; slot[1] = slot[2]; slot[2] = t;
            enxt = ef1;
          }
          // the next column's nxt: f2 (accepted) or the current network through x+1
          // (rejected, in the slot of cur, which becomes the nxt slot below)
          have_nxt = true;
          epre = acc ? ef2 : eden;
          if (acc) { int t = slot[0]; slot[0] = slot[3]; slot[3] = t; }
        }
      }
    }
    int t = slot[0]; slot[0] = slot[1]; slot[1] = t;
    ecur = enxt;
  }
}

// ---------------------------------------------------------------------------
// Chains of |Phi|^2, Phi(S) = Psi(S) + Psi(Sbar) (Sec. II.B): chain ch < n/2
// carries S and chain ch + n/2 its reversal Sbar.  One work-group visits the
// bonds of both in the plain sampler's order; each chain's ratio comes from
// its own environments, and one decision (the S chain's Philox stream) moves
// the same pair in both.  Acceptance |Phi(S')/Phi(S)|^2 with
//   Phi(S')/Phi(S) = (Psi(S) r + Psi(Sbar) rbar) / (Psi(S) + Psi(Sbar)),
// r, rbar the two chains' ratios; Psi(S), Psi(Sbar) are the amplitudes of the
// last top-down contractions (ChainMeta logpsi, sign) multiplied by the ratios
// of every move accepted since, held in registers within a kernel.
// ---------------------------------------------------------------------------
struct PairAmp {
  double la[2];  // log|Psi| of S and Sbar
  double sg[2];  // their signs
};

__device__ inline PairAmp load_pair_amp(const ChainMeta* m0, const ChainMeta* m1) {
  PairAmp A;
  A.la[0] = m0->logpsi;
  A.la[1] = m1->logpsi;
  A.sg[0] = m0->sign < 0 ? -1.0 : 1.0;
  A.sg[1] = m1->sign < 0 ? -1.0 : 1.0;
  return A;
}

// Every thread of the work-group reads the metas before any thread writes them.
__device__ inline void store_pair_amp(ChainMeta* m0, ChainMeta* m1, const PairAmp& A) {
  __syncthreads();
  if (threadIdx.x == 0) {
    m0->logpsi = A.la[0];
    m1->logpsi = A.la[1];
    m0->sign = A.sg[0] < 0.0 ? -1 : 1;
    m1->sign = A.sg[1] < 0.0 ? -1 : 1;
  }
}

__device__ inline void raise_pair(ChainMeta* m0, ChainMeta* m1, int f) {
  raise_flag(m0, f);
  raise_flag(m1, f);
}

__device__ inline bool pair_metropolis(const LatDev& L, int ch, ChainMeta* m0, ChainMeta* m1, PairAmp& A,
                                       const double* num, const double* den, const int* esum, int bond) {
  double r[2];
  for (int c = 0; c < 2; ++c) {
    if (den[c] == 0.0) {
      raise_pair(m0, m1, FLAG_ZERO);
      return false;
    }
    r[c] = scaled(num[c] / den[c], esum[c]);
    if (!isfinite(r[c])) {
      raise_pair(m0, m1, FLAG_NONFINITE);
      return false;
    }
  }
  // amplitudes relative to exp(max log|Psi|): no exponential overflows
  const double mx = fmax(A.la[0], A.la[1]);
  const double pa = A.sg[0] * exp(A.la[0] - mx);
  const double pb = A.sg[1] * exp(A.la[1] - mx);
  const double phi = pa + pb;
  if (phi == 0.0) {
    raise_pair(m0, m1, FLAG_ZERO);
    return false;
  }
  const double q = (pa * r[0] + pb * r[1]) / phi;
  const double R = q * q;
  if (!isfinite(R)) {
    raise_pair(m0, m1, FLAG_NONFINITE);
    return false;
  }
  U64x4 w = philox4x64_10((uint64_t)ch, (uint64_t)m0->sweep, (uint64_t)bond, TAG_METRO, L.seed, (uint64_t)L.lat_id);
  const bool acc = uniform53(w.v[0]) < R;
  if (L.trace && threadIdx.x == 0) {
    double* t = L.trace + 2 * ((int64_t)ch * L.n_bonds + bond);
    t[0] = q;
    t[1] = acc ? 1.0 : 0.0;
  }
  if (acc)
    for (int c = 0; c < 2; ++c)
      if (r[c] != 0.0) {
        A.sg[c] = r[c] < 0.0 ? -A.sg[c] : A.sg[c];
        A.la[c] += log(fabs(r[c]));
      } else {
        A.la[c] = -INFINITY;
      }
  return acc;
}

// Thread 0 counts the proposal in both chains and, if accepted, exchanges the
// pair (k1, k2) in both; the work-group then sees the new spins.
__device__ inline void pair_apply(ChainMeta* m0, ChainMeta* m1, int8_t* sp0, int8_t* sp1, int k1, int k2, bool acc) {
  if (threadIdx.x == 0) {
    m0->proposed += 1;
    m1->proposed += 1;
    if (acc) {
      int8_t a = sp0[k1]; sp0[k1] = sp0[k2]; sp0[k2] = a;
      a = sp1[k1]; sp1[k1] = sp1[k2]; sp1[k2] = a;
      m0->accepted += 1;
      m1->accepted += 1;
    }
  }
  __syncthreads();
}

// Horizontal bonds of row y for the pair (ch, ch + n/2); the last row also
// gives both amplitudes afresh.
template <typename T, int DD, int CC, bool BF16>
__device__ __forceinline__ void ph_hsweep_pair(const LatDev& L, int ch, int y, int last_row, char* tiles) {
  Chain<T> C[2] = {chain_of<T>(L, ch), chain_of<T>(L, ch + L.n_chains / 2)};
  if (chain_flagged(C[0].meta) || chain_flagged(C[1].meta)) return;
  PairAmp A = load_pair_amp(C[0].meta, C[1].meta);
  const int sz = e3sz(L);
  int slot[2][4] = {{0, 1, 2, 3}, {0, 1, 2, 3}};  // cur, nxt, f1, f2 per chain
  int ecur[2] = {0, 0};
  for (int c = 0; c < 2; ++c) set_unit<T>(C[c].ws + L.oT3 + slot[c][0] * sz, sz);
  for (int x = 0; x < L.Lx - 1; ++x) {
    const int k = y * L.Lx + x;
    const int bond = y * (2 * L.Lx - 1) + x;
    const bool anti = C[0].sp[k] != C[0].sp[k + 1];  // the same pair of Sbar is antiparallel too
    if (!anti) trace_skip(L, C[0].id, bond);
    int enxt[2], ef1[2], esum[2];
    double num[2], den[2];
    for (int c = 0; c < 2; ++c) {
      T* tmp = C[c].ws + L.oT3;
      const T* R = C[c].ws + L.oR3;
      const int* eR = C[c].iw + L.ieR3;
      const T* Ux = ub<T>(L, C[c], y, x);
      const T* Dx = db<T>(L, C[c], y + 1, x);
      T* cur = tmp + slot[c][0] * sz;
      T* nxt = tmp + slot[c][1] * sz;
      enxt[c] = ecur[c] + step3<T, DD, CC, BF16>(L, C[c], nxt, cur, y, x, 0, Ux, Dx, false, as_lds(tiles));
      if (anti) {
        T* f1 = tmp + slot[c][2] * sz;
        T* f2 = tmp + slot[c][3] * sz;
        ef1[c] = ecur[c] + step3<T, DD, CC, BF16>(L, C[c], f1, cur, y, x, 1, Ux, Dx, false, as_lds(tiles));
        const int ef2 = ef1[c] + step3<T, DD, CC, BF16>(L, C[c], f2, f1, y, x + 1, 1, ub<T>(L, C[c], y, x + 1),
                                                       db<T>(L, C[c], y + 1, x + 1), false, as_lds(tiles));
        num[c] = wg_dot<T>(f2, R + (int64_t)(x + 2) * sz, sz);
        den[c] = wg_dot<T>(nxt, R + (int64_t)(x + 1) * sz, sz);
        esum[c] = ef2 + eR[x + 2] - enxt[c] - eR[x + 1];
      }
    }
    if (anti) {
      const bool acc = pair_metropolis(L, C[0].id, C[0].meta, C[1].meta, A, num, den, esum, bond);
      pair_apply(C[0].meta, C[1].meta, C[0].sp, C[1].sp, k, k + 1, acc);
      if (acc)  // column x now carries the exchanged tensor: f1 becomes current
        for (int c = 0; c < 2; ++c) {
          int t = slot[c][1]; slot[c][1] = slot[c][2]; slot[c][2] = t;
          enxt[c] = ef1[c];
        }
    }
    for (int c = 0; c < 2; ++c) {
      int t = slot[c][0]; slot[c][0] = slot[c][1]; slot[c][1] = t;
      ecur[c] = enxt[c];
    }
  }
  if (!last_row) {
    store_pair_amp(C[0].meta, C[1].meta, A);
    return;
  }
  const int x = L.Lx - 1;
  for (int c = 0; c < 2; ++c) {
    T* tmp = C[c].ws + L.oT3;
    T* cur = tmp + slot[c][0] * sz;
    T* nxt = tmp + slot[c][1] * sz;
    const int e = ecur[c] + step3<T, DD, CC, BF16>(L, C[c], nxt, cur, y, x, 0, ub<T>(L, C[c], y, x),
                                                  db<T>(L, C[c], y + 1, x), false, as_lds(tiles));
    const double v = (double)nxt[0];
    __syncthreads();  // every thread has read the metas and nxt[0]
    if (threadIdx.x == 0) {
      if (v == 0.0) {
        atomicOr(&C[c].meta->flags, FLAG_ZERO);
      } else if (!isfinite(v)) {
        atomicOr(&C[c].meta->flags, FLAG_NONFINITE);
      } else {
        C[c].meta->logpsi = C[c].dw[L.dlamU + y] + log(fabs(v)) + e * 0.69314718055994530942;
        C[c].meta->sign = v > 0 ? 1 : -1;
      }
    }
  }
}

// Vertical bonds between rows y and y+1 for the pair (ch, ch + n/2).
template <typename T, int DD, int CC, bool BF16>
__device__ __forceinline__ void ph_vsweep_pair(const LatDev& L, int ch, int y, char* lds) {
  Chain<T> C[2] = {chain_of<T>(L, ch), chain_of<T>(L, ch + L.n_chains / 2)};
  if (chain_flagged(C[0].meta) || chain_flagged(C[1].meta)) return;
  PairAmp A = load_pair_amp(C[0].meta, C[1].meta);
  const int sz = e4sz(L);
  int slot[2][3] = {{0, 1, 2}, {0, 1, 2}};  // cur, nxt, f per chain
  int ecur[2] = {0, 0};
  for (int c = 0; c < 2; ++c) set_unit<T>(C[c].ws + L.oT4 + slot[c][0] * sz, sz);
  for (int x = 0; x < L.Lx; ++x) {
    const int k1 = y * L.Lx + x, k2 = (y + 1) * L.Lx + x;
    const int vb = y * (2 * L.Lx - 1) + (L.Lx - 1) + x;
    const bool anti = C[0].sp[k1] != C[0].sp[k2];
    if (!anti) trace_skip(L, C[0].id, vb);
    if (x == L.Lx - 1 && !anti) break;
    int enxt[2], ef[2], esum[2];
    double num[2], den[2];
    for (int c = 0; c < 2; ++c) {
      T* tmp = C[c].ws + L.oT4;
      const T* R = C[c].ws + L.oR4;
      const T* Ux = ub<T>(L, C[c], y, x);
      const T* Dx = db<T>(L, C[c], y + 2, x);
      T* cur = tmp + slot[c][0] * sz;
      T* nxt = tmp + slot[c][1] * sz;
      enxt[c] = ecur[c] + step4<T, DD, CC, BF16>(L, C[c], nxt, cur, y, x, 0, 0, Ux, Dx, false, as_lds(lds));
      if (anti) {
        T* f = tmp + slot[c][2] * sz;
        ef[c] = ecur[c] + step4<T, DD, CC, BF16>(L, C[c], f, cur, y, x, 1, 1, Ux, Dx, false, as_lds(lds));
        num[c] = wg_dot<T>(f, R + (int64_t)(x + 1) * sz, sz);
        den[c] = wg_dot<T>(nxt, R + (int64_t)(x + 1) * sz, sz);
        esum[c] = ef[c] - enxt[c];
      }
    }
    if (anti) {
      const bool acc = pair_metropolis(L, C[0].id, C[0].meta, C[1].meta, A, num, den, esum, vb);
      pair_apply(C[0].meta, C[1].meta, C[0].sp, C[1].sp, k1, k2, acc);
      if (acc)
        for (int c = 0; c < 2; ++c) {
          int t = slot[c][1]; slot[c][1] = slot[c][2]; slot[c][2] = t;
          enxt[c] = ef[c];
        }
    }
    for (int c = 0; c < 2; ++c) {
      int t = slot[c][0]; slot[c][0] = slot[c][1]; slot[c][1] = t;
      ecur[c] = enxt[c];
    }
  }
  store_pair_amp(C[0].meta, C[1].meta, A);
}

// Boundary compression (App. B) of row y into U_y (upper = 1) or D_y.
//
// The canonical SVD compression is computed through Gram matrices: the
// left-to-right QR sweep of its definition only enters through the Gram
// matrices G_j of the left blocks (R_j^T R_j = G_j), which a 2-row column step
// carries exactly; the right-to-left SVD at site j is the eigendecomposition
// of Y^T G_{j-1} Y with Y = (site j) x (right carry), whose leading k_j
// eigenvectors are the kept right singular vectors.  The output state is the
// same; the sign and gauge of every site may differ.  All of it runs in float64
// (the Gram matrices square the condition number of the left blocks).
// LDS of a compression: the Gram step, the GEMM tiles and the eigensolver share it.
template <typename T, int DD, int CC>
constexpr size_t compress_lds() {
  constexpr size_t kGram = env4_lds<double, T, DD, CC, true>();
  constexpr size_t kEig = EIG_LDS_BYTES > GEMM_TILE_BYTES ? EIG_LDS_BYTES : GEMM_TILE_BYTES;
  return kGram > kEig ? kGram : kEig;
}

// LDS of the variational fit: its 3-line steps, the optimal-site step and the GEMM tiles.
template <typename T, int DD, int CC>
constexpr size_t fit_lds() {
  return step3_lds<T, DD, CC, false>();
}

// One 3-line column step of the fit's environments <U'|M_y|U_{y-1}> (upper) or
// <D_{y+1}|M_y|D'> (lower, the row's u and d legs swapped in st): A is the
// input boundary site, U the fitted one in the lower position.  Left step
// Lout[b][r][e] = sum Lin[a][l][c] A[a][x][b] t[l][x][r][y] U[c][y][e]; the
// right step mirrors it.  Returns the power of two taken out.
template <typename T, int DD, int CC>
__device__ inline int fit_env(const LatDev& L, const Chain<T>& C, T* out, const T* in, const T* A, const T* t, S4 st,
                              const T* U, bool right, lds_char* lds) {
  if constexpr (fused3<T, DD, CC>()) {
    if (right)
      env3_fused<T, DD, CC>(out, in, A, sb_mirror(CC, DD), t, st_mirror(st), U, sb_mirror(CC, DD), (char*)lds);
    else
      env3_fused<T, DD, CC>(out, in, A, sb_std(CC, DD), t, st, U, sb_std(CC, DD), (char*)lds);
    return wg_renorm<T>(out, CC * DD * CC);
  }
  if (right)
    env3_step<T>(out, in, A, sb_mirror(L.c, L.d), t, st_mirror(st), U, sb_mirror(L.c, L.d), C.ws + L.oX0,
                 C.ws + L.oX1, L.c, L.d, (char*)lds);
  else
    env3_step<T>(out, in, A, sb_std(L.c, L.d), t, st, U, sb_std(L.c, L.d), C.ws + L.oX0, C.ws + L.oX1, L.c, L.d,
                 (char*)lds);
  return wg_renorm<T>(out, e3sz(L));
}

// The optimal fitted site given orthonormal neighbours:
// Mc[k][y][k'] = sum Lj[a][l][k] A[a][x][b] t[l][x][r][y] Rn[b][r][k'],
// as Y = (A t Rn) (the compression's right half) and Mc = Lj^T Y.
template <typename T, int DD, int CC>
__device__ inline void fit_center(const LatDev& L, const Chain<T>& C, T* Mc, const T* Lj, const T* A, const T* t,
                                  S4 st, const T* Rn, lds_char* lds) {
  if constexpr (fused3<T, DD, CC>()) {
    env3_center_fused<T, DD, CC>(Mc, Lj, A, sb_std(CC, DD), t, st, Rn, (char*)lds);
    return;
  }
  const int c = L.c, d = L.d;
  T* Y = C.ws + L.oX1;
  compress_y<T, T>(Y, A, sb_std(c, d), t, st, Rn, C.ws + L.oX0, c, d, lds);
  wg_gemm_t<T>((char*)lds, Mc, rowmajor(d * c), Lj, colmajor(c), Y, rowmajor(d * c), c, d * c, c * d);
}

// Variational fit (App. B) of row y into U_y (upper = 1) or D_y: minimise the
// distance between the fitted MPS and M_y|U_{y-1}> (or <D_{y+1}|M_y) by
// L.fit_sweeps sweeps of single-site updates, in the working precision.
//   start: leading kl x kr blocks of the product sites, brought to
//          right-orthonormal form from the right (LQ, factor into the left
//          neighbour); right environments of the start;
//   sweep: left to right, the optimal site Lj B Rn replaced by its QR's Q and
//          the left environment advanced; right to left, the same replaced by
//          its LQ's orthonormal rows and the right environment advanced;
//   end:   the optimal site 0 normalised; its norm (with the environments'
//          powers of two) goes into the log-scale.
// Bond dimensions are the plan's (those of the canonical compression).
template <typename T, int DD, int CC>
__device__ __forceinline__ void ph_compress_var(const LatDev& L, int ch, int y, int upper, char* lds) {
  Chain<T> C = chain_of<T>(L, ch);
  if (chain_flagged(C.meta)) return;
  const int c = L.c, d = L.d, Lx = L.Lx, ssz = c * d * c;
  const int in_slot = upper ? y : y + 1;
  const int out_slot = upper ? y + 1 : y;
  auto A_in = [&](int x) -> const T* { return upper ? ub<T>(L, C, in_slot, x) : db<T>(L, C, in_slot, x); };
  auto A_out = [&](int x) -> T* { return upper ? ub<T>(L, C, out_slot, x) : db<T>(L, C, out_slot, x); };
  auto tsite = [&](int x) -> const T* { const int k = y * Lx + x; return tw<T>(L, k, C.sp[k]); };
  auto phys = [&](int x) { const int k = y * Lx + x; return upper ? L.dims[4 * k + 3] : L.dims[4 * k + 1]; };
  const int32_t* kb = upper ? (L.kU + (y + 1) * (Lx + 1)) : (L.kD + y * (Lx + 1));
  const S4 st = upper ? st_std(d) : st_swapud(st_std(d));
  T* Le = C.ws + L.oL3;
  T* Re = C.ws + L.oR3;
  int* eL = C.iw + L.ieL3;
  int* eR = C.iw + L.ieR3;
  T* Mc = C.ws + L.oT3;
  T* Xq = Mc + ssz;        // QR scratch: the factored matrix (R in its upper triangle)
  T* Qq = Xq + ssz;        // QR scratch: Q; also the carry's temporary
  lds_char* ll = as_lds(lds);
  // the fitted site x as a (k_x p) x k_{x+1} matrix (QR), or its transpose (LQ)
  auto qr_view = [&](int x) { return view(phys(x), d * c, c, 1, 1, 0); };
  auto lq_view = [&](int x) { return view(kb[x + 1], c, 1, 1, d * c, 0); };

  // start
  for (int x = 0; x < Lx; ++x) {
    const int k = y * Lx + x;
    fit_start<T>(A_out(x), A_in(x), sb_std(c, d), tsite(x), st, c, d, kb[x], kb[x + 1], phys(x), L.dims[4 * k],
                 L.dims[4 * k + 2]);
  }
  for (int x = Lx - 1; x >= 1; --x) {
    const int m = phys(x) * kb[x + 1], n = kb[x];
    fit_qr_any<T>(A_out(x), ssz, lq_view(x), m, n, Xq, Qq);
    fit_carry<T>(A_out(x - 1), Xq, m, n, kb[x - 1], phys(x - 1), c, d, Qq);
  }
  set_unit<T>(Re + (int64_t)Lx * ssz, ssz);
  set_unit<T>(Le, ssz);
  if (threadIdx.x == 0) { eR[Lx] = 0; eL[0] = 0; }
  __syncthreads();
  for (int x = Lx - 1; x >= 1; --x) {
    const int e = fit_env<T, DD, CC>(L, C, Re + (int64_t)x * ssz, Re + (int64_t)(x + 1) * ssz, A_in(x), tsite(x), st,
                                     A_out(x), true, ll);
    if (threadIdx.x == 0) eR[x] = eR[x + 1] + e;
    __syncthreads();
  }
  for (int s = 0; s < L.fit_sweeps; ++s) {
    for (int x = 0; x < Lx - 1; ++x) {
      fit_center<T, DD, CC>(L, C, Mc, Le + (int64_t)x * ssz, A_in(x), tsite(x), st, Re + (int64_t)(x + 1) * ssz, ll);
      wg_copy<T>(A_out(x), Mc, ssz);
      fit_qr_any<T>(A_out(x), ssz, qr_view(x), kb[x] * phys(x), kb[x + 1], Xq, Qq);
      const int e = fit_env<T, DD, CC>(L, C, Le + (int64_t)(x + 1) * ssz, Le + (int64_t)x * ssz, A_in(x), tsite(x),
                                       st, A_out(x), false, ll);
      if (threadIdx.x == 0) eL[x + 1] = eL[x] + e;
      __syncthreads();
    }
    for (int x = Lx - 1; x >= 1; --x) {
      fit_center<T, DD, CC>(L, C, Mc, Le + (int64_t)x * ssz, A_in(x), tsite(x), st, Re + (int64_t)(x + 1) * ssz, ll);
      wg_copy<T>(A_out(x), Mc, ssz);
      fit_qr_any<T>(A_out(x), ssz, lq_view(x), phys(x) * kb[x + 1], kb[x], Xq, Qq);
      const int e = fit_env<T, DD, CC>(L, C, Re + (int64_t)x * ssz, Re + (int64_t)(x + 1) * ssz, A_in(x), tsite(x),
                                       st, A_out(x), true, ll);
      if (threadIdx.x == 0) eR[x] = eR[x + 1] + e;
      __syncthreads();
    }
  }
  // site 0: the optimal tensor with everything to its right orthonormal
  fit_center<T, DD, CC>(L, C, Mc, Le, A_in(0), tsite(0), st, Re + ssz, ll);
  double nrm2 = 0.0;
  for (int i = threadIdx.x; i < ssz; i += WG) nrm2 += (double)Mc[i] * (double)Mc[i];
  nrm2 = wg_sum(nrm2);
  const double nu = sqrt(nrm2);
  const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
  T* out0 = A_out(0);
  for (int i = threadIdx.x; i < ssz; i += WG) out0[i] = (T)((double)Mc[i] * inv);
  if (threadIdx.x == 0) {
    if (!(nu > 0.0)) atomicOr(&C.meta->flags, FLAG_ZERO);
    else if (!isfinite(nu)) atomicOr(&C.meta->flags, FLAG_NONFINITE);
    const double lognu = log(nu) + eR[1] * 0.69314718055994530942;
    if (upper) C.dw[L.dlamU + y + 1] = C.dw[L.dlamU + y] + lognu;
    else C.dw[L.dlamD + y] = C.dw[L.dlamD + y + 1] + lognu;
  }
  __syncthreads();
}

template <typename T, int DD, int CC>
__device__ __forceinline__ void ph_compress(const LatDev& L, int ch, int y, int upper, char* lds) {
  Chain<T> C = chain_of<T>(L, ch);
  if (chain_flagged(C.meta)) return;
  double* cw = L.cws + (int64_t)ch * L.cws_stride;
  const int c = L.c, d = L.d, Lx = L.Lx;
  const int ssz = c * d * c, gsz = c * d * d * c;
  const int in_slot = upper ? y : y + 1;
  const int out_slot = upper ? y + 1 : y;
  auto A_in = [&](int x) -> const T* { return upper ? ub<T>(L, C, in_slot, x) : db<T>(L, C, in_slot, x); };
  auto A_out = [&](int x) -> T* { return upper ? ub<T>(L, C, out_slot, x) : db<T>(L, C, out_slot, x); };
  const int32_t* kout = upper ? (L.kU + (y + 1) * (Lx + 1)) : (L.kD + y * (Lx + 1));
  const S3 sA = sb_std(c, d);
  const S4 st = upper ? st_std(d) : st_swapud(st_std(d));
  const S4 st2 = st_swapud(st);
  double* G = cw + L.cG;
  double* X0 = cw + L.cX0;
  double* X1 = cw + L.cX1;
  // Gram matrices of the left blocks: G[0] = G_{-1} (unit), G[j+1] = G_j.
  set_unit<double>(G, gsz);
  for (int j = 0; j < Lx - 1; ++j) {
    const int k = y * Lx + j;
    const T* t = tw<T>(L, k, C.sp[k]);
    if constexpr (DD > 0)
      env4_fused<double, T, DD, CC, true>(G + (int64_t)(j + 1) * gsz, G + (int64_t)j * gsz, A_in(j), sA, t, st,
                                          t, st2, A_in(j), sA, lds);
    else
      env4_step<double, T>(G + (int64_t)(j + 1) * gsz, G + (int64_t)j * gsz, A_in(j), sA, t, st, t, st2, A_in(j),
                           sA, X0, X1, c, d, lds);
    wg_renorm<double>(G + (int64_t)(j + 1) * gsz, gsz);
  }
  double* Ta = cw + L.cTa;
  double* Tb = cw + L.cTb;
  double* Y = cw + L.cY;
  double* W = cw + L.cW;
  double* H = cw + L.cH;
  double* Hc = cw + L.cHc;
  double* Vk = cw + L.cVk;
  double* Vp = cw + L.cVp;
  set_unit<double>(Ta, ssz);
  int eT = 0;
  const int dc = d * c;
  for (int j = Lx - 1; j >= 1; --j) {
    const int k = y * Lx + j;
    const T* t = tw<T>(L, k, C.sp[k]);
    compress_y<double, T>(Y, A_in(j), sA, t, st, Ta, X0, c, d, as_lds(lds));
    // W = G_{j-1} Y, G viewed as ((a,l), (a',l')); stored [a'][a][l][l'] (fused) or [a][l][l'][a']
    const View gv = DD > 0 ? view(d, d * d, d, d, c * d * d, 1) : view(d, d * d * c, d * c, d, 1, c);
    wg_gemm_t<double>(lds, W, rowmajor(dc), G + (int64_t)j * gsz, gv, Y, rowmajor(dc), dc, dc, dc);
    // H = Y^T W
    wg_gemm_t<double>(lds, H, rowmajor(dc), Y, colmajor(dc), W, rowmajor(dc), dc, dc, dc);
    const int p = upper ? L.dims[4 * k + 3] : L.dims[4 * k + 1];
    const int kr = kout[j + 1], kl = kout[j];
    const int n = p * kr;
    // compact n x n problem over the valid (dd, kk) pairs
    for (int i = threadIdx.x; i < n * n; i += WG) {
      int a = i / n, b = i - a * n;
      Hc[i] = H[((a / kr) * c + a % kr) * dc + (b / kr) * c + b % kr];
    }
    __syncthreads();
    sym_topk_eig(Hc, n, kl, Vk, cw + L.cLam, cw + L.cRefl, lds);
    // new site j: rows k' < kl are the kept eigenvectors, in descending order
    for (int i = threadIdx.x; i < ssz; i += WG) Vp[i] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < n * kl; i += WG) {
      int q = i / kl, r = i - q * kl;
      Vp[r * dc + (q / kr) * c + q % kr] = Vk[i];
    }
    __syncthreads();
    T* out = A_out(j);
    for (int i = threadIdx.x; i < ssz; i += WG) out[i] = (T)Vp[i];
    // carry: Tb[(a,l)][k'] = sum_{(dd,kk)} Y[(a,l)][(dd,kk)] Vp[k'][(dd,kk)]
    wg_gemm_t<double>(lds, Tb, rowmajor(c), Y, rowmajor(dc), Vp, colmajor(dc), dc, c, dc);
    eT += wg_renorm<double>(Tb, ssz);
    double* tt = Ta; Ta = Tb; Tb = tt;
  }
  {
    const int k = y * Lx;
    const T* t = tw<T>(L, k, C.sp[k]);
    compress_y<double, T>(Y, A_in(0), sA, t, st, Ta, X0, c, d, as_lds(lds));
    double nrm2 = 0.0;
    for (int i = threadIdx.x; i < dc; i += WG) nrm2 += Y[i] * Y[i];
    nrm2 = wg_sum(nrm2);
    double nu = sqrt(nrm2);
    T* out = A_out(0);
    double inv = nu > 0 ? 1.0 / nu : 0.0;
    for (int i = threadIdx.x; i < ssz; i += WG) out[i] = (i < dc) ? (T)(Y[i] * inv) : T(0);
    if (threadIdx.x == 0) {
      if (!(nu > 0.0)) atomicOr(&C.meta->flags, FLAG_ZERO);
      else if (!isfinite(nu)) atomicOr(&C.meta->flags, FLAG_NONFINITE);
      double lognu = log(nu) + eT * 0.69314718055994530942;
      if (upper) C.dw[L.dlamU + y + 1] = C.dw[L.dlamU + y] + lognu;
      else C.dw[L.dlamD + y] = C.dw[L.dlamD + y + 1] + lognu;
    }
    __syncthreads();
  }
}

// Measurement of row y (App. C): log-derivatives of its sites and its
// horizontal pair ratios, all from the cached left/right auxiliary tensors.
template <typename T, int DD, int CC>
__device__ __forceinline__ void ph_measure3(const LatDev& L, int ch, int y, const SampleOut& o, char* tiles) {
  Chain<T> C = chain_of<T>(L, ch);
  if (chain_flagged(C.meta)) return;
  const int sz = e3sz(L), Lx = L.Lx, d = L.d;
  T* R = C.ws + L.oR3;
  T* Le = C.ws + L.oL3;
  T* tmp = C.ws + L.oT3;
  int* eR = C.iw + L.ieR3;
  int* eL = C.iw + L.ieL3;
  set_unit<T>(R + (int64_t)Lx * sz, sz);
  set_unit<T>(Le, sz);
  if (threadIdx.x == 0) { eR[Lx] = 0; eL[0] = 0; }
  __syncthreads();
  for (int x = Lx - 1; x >= 1; --x) {
    int e = step3<T, DD, CC>(L, C, R + (int64_t)x * sz, R + (int64_t)(x + 1) * sz, y, x, 0, ub<T>(L, C, y, x),
                     db<T>(L, C, y + 1, x), true, as_lds(tiles));
    if (threadIdx.x == 0) eR[x] = eR[x + 1] + e;
    __syncthreads();
  }
  // left environments Le[1..max(Lx-1,1)]; Le[Lx] of a wider row is never needed
  for (int x = 0; x < (Lx > 1 ? Lx - 1 : 1); ++x) {
    int e = step3<T, DD, CC>(L, C, Le + (int64_t)(x + 1) * sz, Le + (int64_t)x * sz, y, x, 0, ub<T>(L, C, y, x),
                     db<T>(L, C, y + 1, x), false, as_lds(tiles));
    if (threadIdx.x == 0) eL[x + 1] = eL[x] + e;
    __syncthreads();
  }
  const double Nm = wg_dot<T>(Le + sz, R + sz, sz);
  const int eN = eL[1] + eR[1];
  if (Nm == 0.0) { raise_flag(C.meta, FLAG_ZERO); return; }
  if (o.psi_meas && y == L.Ly - 1 && threadIdx.x == 0) {
    // the bottom row's network is Psi itself (D_{Ly} trivial)
    C.meta->logpsi = C.dw[L.dlamU + y] + log(fabs(Nm)) + eN * 0.69314718055994530942;
    C.meta->sign = Nm > 0 ? 1 : -1;
  }
  if (o.dlnpsi) {
    T* Dl = C.ws + L.oDl;
    for (int x = 0; x < Lx; ++x) {
      const int k = y * Lx + x;
      if constexpr (fused3<T, DD, CC>())
        defect3_fused<T, DD, CC>(Dl, Le + (int64_t)x * sz, ub<T>(L, C, y, x), sb_std(CC, DD),
                                 R + (int64_t)(x + 1) * sz, db<T>(L, C, y + 1, x), sb_std(CC, DD), tiles);
      else
        defect3<T>(Dl, Le + (int64_t)x * sz, ub<T>(L, C, y, x), sb_std(L.c, d), R + (int64_t)(x + 1) * sz,
                   db<T>(L, C, y + 1, x), sb_std(L.c, d), C.ws + L.oX0, C.ws + L.oX1, L.c, d, as_lds(tiles));
      const double f = ldexp(1.0 / Nm, eL[x] + eR[x + 1] - eN);
      const int dl = L.dims[4 * k], du = L.dims[4 * k + 1], dr = L.dims[4 * k + 2], dd = L.dims[4 * k + 3];
      const int n = dl * du * dr * dd;
      T* outp = (T*)o.dlnpsi + ((int64_t)ch * o.n_meas + meas_index(o, C.meta)) * o.np_half + L.coff[k];
      for (int i = threadIdx.x; i < n; i += WG) {
        int l = i / (du * dr * dd), u = (i / (dr * dd)) % du, r = (i / dd) % dr, q = i % dd;
        outp[i] = (T)((double)Dl[((l * d + u) * d + r) * d + q] * f);
      }
      __syncthreads();
    }
  }
  double eacc = 0.0;
  for (int x = 0; x < Lx - 1; ++x) {
    const int k = y * Lx + x;
    const int pair = y * (Lx - 1) + x;
    double rho = 0.0;
    if (C.sp[k] == C.sp[k + 1]) {
      eacc += 0.25 * L.J1;
    } else {
      int e1 = eL[x] + step3<T, DD, CC>(L, C, tmp, Le + (int64_t)x * sz, y, x, 1, ub<T>(L, C, y, x), db<T>(L, C, y + 1, x),
                                false, as_lds(tiles));
      int e2 = e1 + step3<T, DD, CC>(L, C, tmp + sz, tmp, y, x + 1, 1, ub<T>(L, C, y, x + 1), db<T>(L, C, y + 1, x + 1),
                             false, as_lds(tiles));
      double num = wg_dot<T>(tmp + sz, R + (int64_t)(x + 2) * sz, sz);
      rho = ldexp(num / Nm, e2 + eR[x + 2] - eN);
      eacc += -0.25 * L.J1 + 0.5 * L.J1 * rho;
    }
    if (o.ratios && threadIdx.x == 0) o.ratios[(int64_t)ch * o.n_pairs + pair] = rho;
  }
  if (threadIdx.x == 0) {
    if (!isfinite(eacc)) atomicOr(&C.meta->flags, FLAG_NONFINITE);
    C.meta->e_acc += eacc;
  }
}

// Vertical and diagonal pairs between rows y and y+1 (two-row network).
template <typename T, int DD, int CC, int BBX = 0>
__device__ __forceinline__ void ph_measure4(const LatDev& L, int ch, int y, const SampleOut& o, char* lds) {
  Chain<T> C = chain_of<T>(L, ch);
  if (chain_flagged(C.meta)) return;
  const int sz = e4sz(L), Lx = L.Lx;
  T* R = C.ws + L.oR4;
  T* Le = C.ws + L.oL4;
  T* tmp = C.ws + L.oT4;
  int* eR = C.iw + L.ieR4;
  int* eL = C.iw + L.ieL4;
  set_unit<T>(R + (int64_t)Lx * sz, sz);
  set_unit<T>(Le, sz);
  if (threadIdx.x == 0) { eR[Lx] = 0; eL[0] = 0; }
  __syncthreads();
  for (int x = Lx - 1; x >= 1; --x) {
    int e = step4<T, DD, CC, false, BBX>(L, C, R + (int64_t)x * sz, R + (int64_t)(x + 1) * sz, y, x, 0, 0, ub<T>(L, C, y, x),
                     db<T>(L, C, y + 2, x), true, as_lds(lds));
    if (threadIdx.x == 0) eR[x] = eR[x + 1] + e;
    __syncthreads();
  }
  // left environments Le[1..max(Lx-1,1)]; Le[Lx] of a wider row pair is never needed
  for (int x = 0; x < (Lx > 1 ? Lx - 1 : 1); ++x) {
    int e = step4<T, DD, CC, false, BBX>(L, C, Le + (int64_t)(x + 1) * sz, Le + (int64_t)x * sz, y, x, 0, 0, ub<T>(L, C, y, x),
                     db<T>(L, C, y + 2, x), false, as_lds(lds));
    if (threadIdx.x == 0) eL[x + 1] = eL[x] + e;
    __syncthreads();
  }
  const double Nm = wg_dot<T>(Le + sz, R + sz, sz);
  const int eN = eL[1] + eR[1];
  if (Nm == 0.0) { raise_flag(C.meta, FLAG_ZERO); return; }
  double eacc = 0.0;
  const int base_v = L.Ly * (Lx - 1);
  for (int x = 0; x < Lx; ++x) {
    const int k1 = y * Lx + x, k2 = (y + 1) * Lx + x;
    double rho = 0.0;
    if (L.J1 == 0.0) {
      // no nearest-neighbour terms (the knight-bond evaluation of a transposed lattice)
    } else if (C.sp[k1] == C.sp[k2]) {
      eacc += 0.25 * L.J1;
    } else {
      int e1 = eL[x] + step4<T, DD, CC, false, BBX>(L, C, tmp, Le + (int64_t)x * sz, y, x, 1, 1, ub<T>(L, C, y, x), db<T>(L, C, y + 2, x), false, as_lds(lds));
      double num = wg_dot<T>(tmp, R + (int64_t)(x + 1) * sz, sz);
      rho = ldexp(num / Nm, e1 + eR[x + 1] - eN);
      eacc += -0.25 * L.J1 + 0.5 * L.J1 * rho;
    }
    if (o.ratios && threadIdx.x == 0) o.ratios[(int64_t)ch * o.n_pairs + base_v + y * Lx + x] = rho;
  }
  if (L.Jd != 0.0 || L.Ja != 0.0) {
    const int base_d = base_v + (L.Ly - 1) * Lx;
    for (int x = 0; x < Lx - 1; ++x) {
      for (int which = 0; which < 2; ++which) {
        // which 0: (y,x)-(y+1,x+1); which 1: (y,x+1)-(y+1,x)
        const int kp = which == 0 ? y * Lx + x : y * Lx + x + 1;
        const int kq = which == 0 ? (y + 1) * Lx + x + 1 : (y + 1) * Lx + x;
        const double Jw = which == 0 ? L.Jd : L.Ja;
        double rho = 0.0;
        if (Jw == 0.0) {
          // an uncoupled diagonal (triangular lattice): no term, ratio slot 0
        } else if (C.sp[kp] == C.sp[kq]) {
          eacc += 0.25 * Jw;
        } else {
          // column x: flips (y,x) for which 0 and (y+1,x) for which 1; column x+1 the other site
          int f1a = which == 0 ? 1 : 0, f1b = which == 0 ? 0 : 1;
          int e1 = eL[x] + step4<T, DD, CC, false, BBX>(L, C, tmp, Le + (int64_t)x * sz, y, x, f1a, f1b, ub<T>(L, C, y, x),
                                    db<T>(L, C, y + 2, x), false, as_lds(lds));
          int e2 = e1 + step4<T, DD, CC, false, BBX>(L, C, tmp + sz, tmp, y, x + 1, 1 - f1a, 1 - f1b, ub<T>(L, C, y, x + 1),
                                 db<T>(L, C, y + 2, x + 1), false, as_lds(lds));
          double num = wg_dot<T>(tmp + sz, R + (int64_t)(x + 2) * sz, sz);
          rho = ldexp(num / Nm, e2 + eR[x + 2] - eN);
          eacc += -0.25 * Jw + 0.5 * Jw * rho;
        }
        if (o.ratios && threadIdx.x == 0)
          o.ratios[(int64_t)ch * o.n_pairs + base_d + 2 * (y * (Lx - 1) + x) + which] = rho;
      }
    }
  }
  if (L.Jk != 0.0) {
    // knight bonds (y,x)-(y+1,x+2) of the triangular lattice: the 2-row network with
    // site (y,x) flipped in column x, column x+1 unchanged and (y+1,x+2) flipped in column x+2
    const int base_k = base_v + (L.Ly - 1) * Lx + ((L.Jd != 0.0 || L.Ja != 0.0) ? 2 * (L.Ly - 1) * (Lx - 1) : 0);
    for (int x = 0; x + 2 < Lx; ++x) {
      const int kp = y * Lx + x, kq = (y + 1) * Lx + x + 2;
      double rho = 0.0;
      if (C.sp[kp] == C.sp[kq]) {
        eacc += 0.25 * L.Jk;
      } else {
        int e = eL[x] + step4<T, DD, CC, false, BBX>(L, C, tmp, Le + (int64_t)x * sz, y, x, 1, 0, ub<T>(L, C, y, x),
                                                     db<T>(L, C, y + 2, x), false, as_lds(lds));
        e += step4<T, DD, CC, false, BBX>(L, C, tmp + sz, tmp, y, x + 1, 0, 0, ub<T>(L, C, y, x + 1),
                                         db<T>(L, C, y + 2, x + 1), false, as_lds(lds));
        e += step4<T, DD, CC, false, BBX>(L, C, tmp + 2 * sz, tmp + sz, y, x + 2, 0, 1, ub<T>(L, C, y, x + 2),
                                         db<T>(L, C, y + 2, x + 2), false, as_lds(lds));
        const double num = wg_dot<T>(tmp + 2 * sz, R + (int64_t)(x + 3) * sz, sz);
        rho = ldexp(num / Nm, e + eR[x + 3] - eN);
        eacc += -0.25 * L.Jk + 0.5 * L.Jk * rho;
      }
      if (o.ratios && threadIdx.x == 0) o.ratios[(int64_t)ch * o.n_pairs + base_k + y * (Lx - 2) + x] = rho;
    }
  }
  if (o.plaq) {
    // flips of the movable plaquettes (y, x): both columns exchanged in both rows
    for (int x = 0; x < Lx - 1; ++x) {
      const int k1 = y * Lx + x, k2 = k1 + Lx;
      double rho = 0.0;
      if (C.sp[k1] + C.sp[k1 + 1] + C.sp[k2] + C.sp[k2 + 1] == 2) {
        int e1 = eL[x] + step4<T, DD, CC, false, BBX>(L, C, tmp, Le + (int64_t)x * sz, y, x, 1, 1, ub<T>(L, C, y, x),
                                          db<T>(L, C, y + 2, x), false, as_lds(lds));
        int e2 = e1 + step4<T, DD, CC, false, BBX>(L, C, tmp + sz, tmp, y, x + 1, 1, 1, ub<T>(L, C, y, x + 1),
                                       db<T>(L, C, y + 2, x + 1), false, as_lds(lds));
        double num = wg_dot<T>(tmp + sz, R + (int64_t)(x + 2) * sz, sz);
        rho = ldexp(num / Nm, e2 + eR[x + 2] - eN);
      }
      if (threadIdx.x == 0) o.plaq[(int64_t)ch * (L.Ly - 1) * (Lx - 1) + y * (Lx - 1) + x] = rho;
    }
  }
  if (threadIdx.x == 0) {
    if (!isfinite(eacc)) atomicOr(&C.meta->flags, FLAG_NONFINITE);
    C.meta->e_acc += eacc;
  }
}

// Wrappers: one work-group per chain, one phase of one row.
template <typename T, int DD, int CC, bool BF16>
__global__ void __launch_bounds__(WG, 2) k_row3_right(LatDev L, int y, int ub_slot, int db_slot) {
  __shared__ __attribute__((aligned(16))) char lds[step3_lds<T, DD, CC, BF16>()];
  ph_row3_right<T, DD, CC, BF16>(L, blockIdx.x, y, ub_slot, db_slot, lds);
}
template <typename T, int DD, int CC, bool BF16>
__global__ void __launch_bounds__(WG, 2) k_hsweep(LatDev L, int y, int last_row, int moves) {
  __shared__ __attribute__((aligned(16))) char lds[step3_lds<T, DD, CC, BF16>()];
  ph_hsweep<T, DD, CC, BF16>(L, blockIdx.x, y, last_row, moves, lds);
}
// LDS of a 2-row step: the bf16 step stages compact bf16 operands.
template <typename T, int DD, int CC, bool BF16, int BBX = 0>
constexpr size_t step4_lds() {
  if constexpr (BF16 && DD > 0) return Env4Bf<DD, CC>::lds_bytes();
  else return env4_lds<T, T, DD, CC, false, BBX>();
}

// The pair sampler's decision phases: one work-group per pair (n/2 of them).
template <typename T, int DD, int CC, bool BF16>
__global__ void __launch_bounds__(WG, 2) k_hsweep_pair(LatDev L, int y, int last_row) {
  __shared__ __attribute__((aligned(16))) char lds[step3_lds<T, DD, CC, BF16>()];
  ph_hsweep_pair<T, DD, CC, BF16>(L, blockIdx.x, y, last_row, lds);
}
// BBX: b-block of the fused 2-row step (a tile variant, 0 = default).
template <typename T, int DD, int CC, bool BF16, int BBX = 0>
__global__ void __launch_bounds__(WG, 2) k_row4_right(LatDev L, int y) {
  __shared__ __attribute__((aligned(16))) char lds[step4_lds<T, DD, CC, BF16, BBX>()];
  ph_row4_right<T, DD, CC, BF16, BBX>(L, blockIdx.x, y, lds);
}
template <typename T, int DD, int CC, bool BF16, bool LEARN, int BBX = 0>
__global__ void __launch_bounds__(WG, 2) k_vsweep(LatDev L, int y) {
  __shared__ __attribute__((aligned(16)))
  char lds[cmax(step4_lds<T, DD, CC, BF16, BBX>(), LEARN ? (BF16 ? net_bf_lds_bytes() : net_lds_bytes<T>()) : 0)];
  ph_vsweep<T, DD, CC, BF16, LEARN, BBX>(L, blockIdx.x, y, lds);
}
template <typename T, int DD, int CC, bool BF16>
__global__ void __launch_bounds__(WG, 2) k_vsweep_pair(LatDev L, int y) {
  __shared__ __attribute__((aligned(16))) char lds[step4_lds<T, DD, CC, BF16>()];
  ph_vsweep_pair<T, DD, CC, BF16>(L, blockIdx.x, y, lds);
}
template <typename T, int DD, int CC>
__global__ void __launch_bounds__(WG, 2) k_compress(LatDev L, int y, int upper) {
  __shared__ __attribute__((aligned(16))) char lds[compress_lds<T, DD, CC>()];
  ph_compress<T, DD, CC>(L, blockIdx.x, y, upper, lds);
}
// The variational fit in a kernel of its own (it needs far less LDS than the
// canonical compression's eigensolver).
template <typename T, int DD, int CC>
__global__ void __launch_bounds__(WG, 2) k_compress_fit(LatDev L, int y, int upper) {
  __shared__ __attribute__((aligned(16))) char lds[fit_lds<T, DD, CC>()];
  ph_compress_var<T, DD, CC>(L, blockIdx.x, y, upper, lds);
}
template <typename T, int DD, int CC>
__global__ void __launch_bounds__(WG, 2) k_measure3(LatDev L, int y, SampleOut o) {
  __shared__ __attribute__((aligned(16))) char lds[step3_lds<T, DD, CC, false, true>()];
  ph_measure3<T, DD, CC>(L, blockIdx.x, y, o, lds);
}
template <typename T, int DD, int CC, int BBX = 0>
__global__ void __launch_bounds__(WG, 2) k_measure4(LatDev L, int y, SampleOut o) {
  __shared__ __attribute__((aligned(16))) char lds[env4_lds<T, T, DD, CC, false, BBX>()];
  ph_measure4<T, DD, CC, BBX>(L, blockIdx.x, y, o, lds);
}

__global__ void k_begin_sample(LatDev L) {
  int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch < L.n_chains) L.meta[ch].e_acc = 0.0;
}

__global__ void k_finish_sample(LatDev L, SampleOut o, int n_active) {
  int ch = blockIdx.x;
  if (ch >= n_active) return;
  const ChainMeta* m = L.meta + ch;
  int64_t idx = (int64_t)ch * o.n_meas + meas_index(o, m);
  if (threadIdx.x == 0) {
    if (o.log_abs_psi) o.log_abs_psi[idx] = m->logpsi;
    if (o.sign) o.sign[idx] = (int8_t)m->sign;
    if (o.e_loc) o.e_loc[idx] = m->e_acc;
  }
  if (o.spins)
    for (int i = threadIdx.x; i < L.N; i += blockDim.x) o.spins[idx * L.N + i] = L.spins[(int64_t)ch * L.N + i];
}

__global__ void k_next_sweep(LatDev L) {
  int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch < L.n_chains) L.meta[ch].sweep += 1;
}

// ---------------------------------------------------------------------------
// Persistent whole-sweep kernel: a work-group takes (lattice, chain) items from
// a queue and runs one complete sweep of that chain -- every phase of the
// top-down sampling pass and (if requested) the bottom-up measurement pass --
// before taking the next.  Chains of lattices of different sizes share one
// launch; items are queued largest lattice first, so the short sweeps fill the
// tail.  The queue counter must be zero at launch; every work-group leaves
// when the queue is exhausted.
// ---------------------------------------------------------------------------
template <typename T, int DD, int CC>
constexpr size_t sweep_lds() {
  return cmax(cmax(cmax(env4_lds<T, T, DD, CC>(), compress_lds<T, DD, CC>()), net_lds_bytes<T>()),
              step3_lds<T, DD, CC, false, true>());
}

// Out-of-line phases of the persistent kernel: each keeps its own register
// allocation instead of the union of all phases.  Their LDS argument is typed
// as LDS, so that the phases inlined into them address it with LDS
// instructions (through a plain pointer they would be flat ones).
template <typename T, int DD, int CC, bool BF16>
__device__ __noinline__ void nl_row3_right(const LatDev& L, int ch, int y, lds_char* lds) {
  ph_row3_right<T, DD, CC, BF16>(L, ch, y, y, y + 1, (char*)lds);
}
template <typename T, int DD, int CC, bool BF16>
__device__ __noinline__ void nl_hsweep(const LatDev& L, int ch, int y, lds_char* lds) {
  ph_hsweep<T, DD, CC, BF16>(L, ch, y, y == L.Ly - 1, 1, (char*)lds);
}
template <typename T, int DD, int CC, bool BF16>
__device__ __noinline__ void nl_row4_right(const LatDev& L, int ch, int y, lds_char* lds) {
  ph_row4_right<T, DD, CC, BF16>(L, ch, y, (char*)lds);
}
template <typename T, int DD, int CC, bool BF16, bool LEARN>
__device__ __noinline__ void nl_vsweep(const LatDev& L, int ch, int y, lds_char* lds) {
  ph_vsweep<T, DD, CC, BF16, LEARN>(L, ch, y, (char*)lds);
}
template <typename T, int DD, int CC>
__device__ __noinline__ void nl_compress(const LatDev& L, int ch, int y, int upper, lds_char* lds) {
  ph_compress<T, DD, CC>(L, ch, y, upper, (char*)lds);
}
template <typename T, int DD, int CC>
__device__ __noinline__ void nl_measure3(const LatDev& L, int ch, int y, const SampleOut& o, lds_char* lds) {
  ph_measure3<T, DD, CC>(L, ch, y, o, (char*)lds);
}
template <typename T, int DD, int CC>
__device__ __noinline__ void nl_measure4(const LatDev& L, int ch, int y, const SampleOut& o, lds_char* lds) {
  ph_measure4<T, DD, CC>(L, ch, y, o, (char*)lds);
}

template <typename T, int DD, int CC, bool BF16>
__device__ void chain_sweep(const LatDev& L, int ch, const SampleOut* o, char* lds) {
  const int Ly = L.Ly;
  for (int y = 0; y < Ly; ++y) {
    nl_row3_right<T, DD, CC, BF16>(L, ch, y, (lds_char*)lds);
    __syncthreads();
    nl_hsweep<T, DD, CC, BF16>(L, ch, y, (lds_char*)lds);
    __syncthreads();
    if (y < Ly - 1) {
      nl_row4_right<T, DD, CC, BF16>(L, ch, y, (lds_char*)lds);
      __syncthreads();
      if (L.learned) nl_vsweep<T, DD, CC, BF16, true>(L, ch, y, (lds_char*)lds);
      else nl_vsweep<T, DD, CC, BF16, false>(L, ch, y, (lds_char*)lds);
      __syncthreads();
      nl_compress<T, DD, CC>(L, ch, y, 1, (lds_char*)lds);
      __syncthreads();
    }
  }
  ChainMeta* m = L.meta + ch;
  if (o && threadIdx.x == 0) m->e_acc = 0.0;
  __syncthreads();
  for (int y = Ly - 1; y >= 0; --y) {
    if (o) {
      nl_measure3<T, DD, CC>(L, ch, y, *o, (lds_char*)lds);
      __syncthreads();
      if (y < Ly - 1) {
        nl_measure4<T, DD, CC>(L, ch, y, *o, (lds_char*)lds);
        __syncthreads();
      }
    }
    if (y >= 1) {
      nl_compress<T, DD, CC>(L, ch, y, 0, (lds_char*)lds);
      __syncthreads();
    }
  }
  if (o) {
    const int64_t idx = (int64_t)ch * o->n_meas + meas_index(*o, m);
    if (threadIdx.x == 0) {
      if (o->log_abs_psi) o->log_abs_psi[idx] = m->logpsi;
      if (o->sign) o->sign[idx] = (int8_t)m->sign;
      if (o->e_loc) o->e_loc[idx] = m->e_acc;
    }
    if (o->spins)
      for (int i = threadIdx.x; i < L.N; i += WG) o->spins[idx * L.N + i] = L.spins[(int64_t)ch * L.N + i];
  }
  if (threadIdx.x == 0) m->sweep += 1;
  __syncthreads();
}

template <typename T, int DD, int CC, bool BF16>
__global__ void __launch_bounds__(WG, 2) k_sweep_queue(const LatDev* __restrict__ lats,
                                                       const SampleOut* __restrict__ outs, int measure,
                                                       const int2* __restrict__ items, int n_items,
                                                       int* __restrict__ next) {
  __shared__ __attribute__((aligned(16))) char lds[sweep_lds<T, DD, CC>()];
  __shared__ int item;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(next, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item);
    __syncthreads();
    if (it >= n_items) break;
    const int2 w = items[it];
    const int li = __builtin_amdgcn_readfirstlane(w.x), ch = __builtin_amdgcn_readfirstlane(w.y);
    chain_sweep<T, DD, CC, BF16>(lats[li], ch, measure ? outs + li : nullptr, lds);
  }
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ void k_init_tensors(double* T, int64_t Np, uint64_t seed, int lat_id, double scale, double perturb) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < Np; p += (int64_t)gridDim.x * blockDim.x) {
    const double two_pi = 6.283185307179586476925286766559;
    U64x4 w = philox4x64_10((uint64_t)p, 0, 0, TAG_INIT, seed, (uint64_t)lat_id);
    double z = sqrt(-2.0 * log(1.0 - uniform53(w.v[0]))) * cos(two_pi * uniform53(w.v[1]));
    double v = scale * z;
    if (perturb != 0.0) {
      U64x4 q = philox4x64_10((uint64_t)p, 0, 0, TAG_PERTURB, seed, (uint64_t)lat_id);
      v += perturb * sqrt(-2.0 * log(1.0 - uniform53(q.v[0]))) * cos(two_pi * uniform53(q.v[1]));
    }
    T[p] = v;
  }
}

// Neel list shuffled by Fisher-Yates (Durstenfeld) with Philox indices.
__global__ void k_init_chains(LatDev L) {
  int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= L.n_chains) return;
  int8_t* s = L.spins + (int64_t)ch * L.N;
  for (int i = 0; i < L.N; ++i) s[i] = (int8_t)(((i / L.Lx) + (i % L.Lx)) & 1);
  for (int i = L.N - 1; i >= 1; --i) {
    U64x4 w = philox4x64_10((uint64_t)ch, 0, (uint64_t)i, TAG_SHUFFLE, L.seed, (uint64_t)L.lat_id);
    uint64_t j = ((w.v[0] >> 11) * (uint64_t)(i + 1)) >> 53;
    int8_t a = s[i]; s[i] = s[j]; s[j] = a;
  }
  ChainMeta* m = L.meta + ch;
  m->sweep = 0; m->accepted = 0; m->proposed = 0; m->flags = 0; m->e_acc = 0.0;
  m->p_accepted = 0; m->p_proposed = 0;
}

__global__ void k_copy_spins(LatDev L, const int8_t* src, int n_cfg) {
  int ch = blockIdx.x;
  if (ch >= n_cfg) return;
  for (int i = threadIdx.x; i < L.N; i += blockDim.x) L.spins[(int64_t)ch * L.N + i] = src[(int64_t)ch * L.N + i];
  if (threadIdx.x == 0) {
    ChainMeta* m = L.meta + ch;
    m->flags = 0; m->e_acc = 0.0;
  }
}

__global__ void k_mean(const double* e, int64_t ns, double* out) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < ns; i += WG) s += e[i];
  s = wg_sum(s);
  if (threadIdx.x == 0) *out = s / (double)ns;
}

// Eq. (5) in the full parameter layout; thread q owns compact entry q of every sample.
template <typename T>
__global__ void k_gradient(const int64_t* offs, const int64_t* coff, const int32_t* sz, int N, const double* e,
                           const T* dl, const int8_t* spins, int64_t ns, int64_t nh, const double* emean,
                           double* grad) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nh) return;
  int lo = 0, hi = N - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (coff[mid] <= q) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  const int64_t local = q - coff[k];
  double a0 = 0, a1 = 0, b0 = 0, b1 = 0;
  for (int64_t i = 0; i < ns; ++i) {
    double g = (double)dl[i * nh + q];
    double ei = e[i];
    if (spins[i * N + k]) { a1 += g * ei; b1 += g; } else { a0 += g * ei; b0 += g; }
  }
  const double E = *emean, inv = 1.0 / (double)ns;
  grad[offs[k] + local] = a0 * inv - b0 * inv * E;
  grad[offs[k] + sz[k] + local] = a1 * inv - b1 * inv * E;
}

__global__ void k_sign_sgd(double* T, const double* g, int64_t Np, double step_len, uint64_t seed, int lat_id,
                           uint64_t step) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < Np; p += (int64_t)gridDim.x * blockDim.x) {
    double gv = g[p];
    if (gv == 0.0) continue;
    U64x4 w = philox4x64_10((uint64_t)p, step, 0, TAG_SGD, seed, (uint64_t)lat_id);
    T[p] -= uniform53(w.v[0]) * step_len * (gv > 0 ? 1.0 : -1.0);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <typename T>
void launch_prepare_tensors(const LatDev& L, const double* Tflat, T* Tw, const int64_t* offs, hipStream_t s) {
  int64_t total = (int64_t)L.N * 2 * L.d * L.d * L.d * L.d;
  int blocks = (int)std::min<int64_t>((total + WG - 1) / WG, 65536);
  hipLaunchKernelGGL(k_prepare_tensors<T>, dim3(blocks), dim3(WG), 0, s, L, Tflat, Tw, offs);
}
template <typename T>
void launch_init_trivial(const LatDev& L, hipStream_t s) {
  hipLaunchKernelGGL(k_init_trivial<T>, dim3(L.n_chains), dim3(WG), 0, s, L);
}
// Compile-time (D, Dc) instantiations of the fused 2-row step; other shapes run the generic path.
#define VP_DISPATCH_DC(KERNEL, T, ...)                                                                 \
  do {                                                                                                 \
    if (L.d == 8 && L.c == 16)                                                                         \
      hipLaunchKernelGGL((KERNEL<T, 8, 16>), dim3(L.n_chains), dim3(WG), 0, s, __VA_ARGS__);           \
    else if (L.d == 6 && L.c == 12)                                                                    \
      hipLaunchKernelGGL((KERNEL<T, 6, 12>), dim3(L.n_chains), dim3(WG), 0, s, __VA_ARGS__);           \
    else if (L.d == 4 && L.c == 8)                                                                     \
      hipLaunchKernelGGL((KERNEL<T, 4, 8>), dim3(L.n_chains), dim3(WG), 0, s, __VA_ARGS__);            \
    else                                                                                               \
      hipLaunchKernelGGL((KERNEL<T, 0, 0>), dim3(L.n_chains), dim3(WG), 0, s, __VA_ARGS__);            \
  } while (0)

// The same with a compile-time operand-precision flag BF (bf16 operands when true).
#define VP_DISPATCH_DC_BF(KERNEL, T, BF, ...)                                                          \
  do {                                                                                                 \
    if (L.d == 8 && L.c == 16)                                                                         \
      hipLaunchKernelGGL((KERNEL<T, 8, 16, BF>), dim3(L.n_chains), dim3(WG), 0, s, __VA_ARGS__);       \
    else if (L.d == 6 && L.c == 12)                                                                    \
      hipLaunchKernelGGL((KERNEL<T, 6, 12, BF>), dim3(L.n_chains), dim3(WG), 0, s, __VA_ARGS__);       \
    else if (L.d == 4 && L.c == 8)                                                                     \
      hipLaunchKernelGGL((KERNEL<T, 4, 8, BF>), dim3(L.n_chains), dim3(WG), 0, s, __VA_ARGS__);        \
    else                                                                                               \
      hipLaunchKernelGGL((KERNEL<T, 0, 0, BF>), dim3(L.n_chains), dim3(WG), 0, s, __VA_ARGS__);        \
  } while (0)

template <typename T>
void launch_row3_right(const LatDev& L, int y, int ub_slot, int db_slot, bool bf16, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    if (bf16) { VP_DISPATCH_DC_BF(k_row3_right, T, true, L, y, ub_slot, db_slot); return; }
  }
  VP_DISPATCH_DC_BF(k_row3_right, T, false, L, y, ub_slot, db_slot);
}
template <typename T>
void launch_hsweep(const LatDev& L, int y, int last_row, bool bf16, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    if (bf16) { VP_DISPATCH_DC_BF(k_hsweep, T, true, L, y, last_row, 1); return; }
  }
  VP_DISPATCH_DC_BF(k_hsweep, T, false, L, y, last_row, 1);
}
template <typename T>
void launch_psi_fixed(const LatDev& L, hipStream_t s) {
  const int y = L.Ly - 1;
  VP_DISPATCH_DC_BF(k_hsweep, T, false, L, y, 1, 0);
}
// Tile variants of the fused float32 / float64 2-row step at D = 8, Dc = 16: the
// b-block BB = Dc/4 (variant 0, the default), Dc/8 (1) or Dc/2 (2).
constexpr int tile_bb(int tile) { return tile == 1 ? 2 : (tile == 2 ? 8 : 0); }

// bf16 operands are taken from float64 storage (VP_BF16 works in float64).
template <typename T>
void launch_row4_right(const LatDev& L, int y, bool bf16, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    if (bf16) { VP_DISPATCH_DC_BF(k_row4_right, T, true, L, y); return; }
  }
  if (L.d == 8 && L.c == 16) {
    const dim3 g(L.n_chains), b(WG);
    if (L.tile == 1) hipLaunchKernelGGL((k_row4_right<T, 8, 16, false, tile_bb(1)>), g, b, 0, s, L, y);
    else if (L.tile == 2) hipLaunchKernelGGL((k_row4_right<T, 8, 16, false, tile_bb(2)>), g, b, 0, s, L, y);
    else hipLaunchKernelGGL((k_row4_right<T, 8, 16, false, 0>), g, b, 0, s, L, y);
    return;
  }
  VP_DISPATCH_DC_BF(k_row4_right, T, false, L, y);
}
#define VP_DISPATCH_DC_VS(T, BF, LR)                                                                   \
  do {                                                                                                 \
    if (L.d == 8 && L.c == 16)                                                                         \
      hipLaunchKernelGGL((k_vsweep<T, 8, 16, BF, LR>), dim3(L.n_chains), dim3(WG), 0, s, L, y);        \
    else if (L.d == 6 && L.c == 12)                                                                    \
      hipLaunchKernelGGL((k_vsweep<T, 6, 12, BF, LR>), dim3(L.n_chains), dim3(WG), 0, s, L, y);        \
    else if (L.d == 4 && L.c == 8)                                                                     \
      hipLaunchKernelGGL((k_vsweep<T, 4, 8, BF, LR>), dim3(L.n_chains), dim3(WG), 0, s, L, y);         \
    else                                                                                               \
      hipLaunchKernelGGL((k_vsweep<T, 0, 0, BF, LR>), dim3(L.n_chains), dim3(WG), 0, s, L, y);         \
  } while (0)
template <typename T>
void launch_vsweep(const LatDev& L, int y, bool bf16, bool learned, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    if (bf16) {
      if (learned) VP_DISPATCH_DC_VS(T, true, true);
      else VP_DISPATCH_DC_VS(T, true, false);
      return;
    }
  }
  if (L.d == 8 && L.c == 16) {
    const dim3 g(L.n_chains), b(WG);
    if (learned) {
      if (L.tile == 1) hipLaunchKernelGGL((k_vsweep<T, 8, 16, false, true, tile_bb(1)>), g, b, 0, s, L, y);
      else if (L.tile == 2) hipLaunchKernelGGL((k_vsweep<T, 8, 16, false, true, tile_bb(2)>), g, b, 0, s, L, y);
      else hipLaunchKernelGGL((k_vsweep<T, 8, 16, false, true, 0>), g, b, 0, s, L, y);
    } else {
      if (L.tile == 1) hipLaunchKernelGGL((k_vsweep<T, 8, 16, false, false, tile_bb(1)>), g, b, 0, s, L, y);
      else if (L.tile == 2) hipLaunchKernelGGL((k_vsweep<T, 8, 16, false, false, tile_bb(2)>), g, b, 0, s, L, y);
      else hipLaunchKernelGGL((k_vsweep<T, 8, 16, false, false, 0>), g, b, 0, s, L, y);
    }
    return;
  }
  if (learned) VP_DISPATCH_DC_VS(T, false, true);
  else VP_DISPATCH_DC_VS(T, false, false);
}

// Pair sampler launches: one work-group per chain pair (grid n_chains / 2).
#define VP_DISPATCH_PAIR(KERNEL, T, BF, ...)                                                           \
  do {                                                                                                 \
    const dim3 g(L.n_chains / 2), b(WG);                                                               \
    if (L.d == 8 && L.c == 16) hipLaunchKernelGGL((KERNEL<T, 8, 16, BF>), g, b, 0, s, __VA_ARGS__);    \
    else if (L.d == 6 && L.c == 12) hipLaunchKernelGGL((KERNEL<T, 6, 12, BF>), g, b, 0, s, __VA_ARGS__); \
    else if (L.d == 4 && L.c == 8) hipLaunchKernelGGL((KERNEL<T, 4, 8, BF>), g, b, 0, s, __VA_ARGS__);  \
    else hipLaunchKernelGGL((KERNEL<T, 0, 0, BF>), g, b, 0, s, __VA_ARGS__);                           \
  } while (0)
template <typename T>
void launch_hsweep_pair(const LatDev& L, int y, int last_row, bool bf16, hipStream_t s) {
  if (L.n_chains < 2) return;
  if constexpr (sizeof(T) == 8) {
    if (bf16) { VP_DISPATCH_PAIR(k_hsweep_pair, T, true, L, y, last_row); return; }
  }
  VP_DISPATCH_PAIR(k_hsweep_pair, T, false, L, y, last_row);
}
template <typename T>
void launch_vsweep_pair(const LatDev& L, int y, bool bf16, hipStream_t s) {
  if (L.n_chains < 2) return;
  if constexpr (sizeof(T) == 8) {
    if (bf16) { VP_DISPATCH_PAIR(k_vsweep_pair, T, true, L, y); return; }
  }
  VP_DISPATCH_PAIR(k_vsweep_pair, T, false, L, y);
}
template <typename T>
void launch_compress(const LatDev& L, int y, int upper, hipStream_t s) {
  if (L.cmode == 1) VP_DISPATCH_DC(k_compress_fit, T, L, y, upper);
  else VP_DISPATCH_DC(k_compress, T, L, y, upper);
}
template <typename T>
void launch_measure3(const LatDev& L, int y, const SampleOut& o, hipStream_t s) {
  VP_DISPATCH_DC(k_measure3, T, L, y, o);
}
template <typename T>
void launch_measure4(const LatDev& L, int y, const SampleOut& o, hipStream_t s) {
  if (L.d == 8 && L.c == 16) {
    const dim3 g(L.n_chains), b(WG);
    if (L.tile == 1) hipLaunchKernelGGL((k_measure4<T, 8, 16, tile_bb(1)>), g, b, 0, s, L, y, o);
    else if (L.tile == 2) hipLaunchKernelGGL((k_measure4<T, 8, 16, tile_bb(2)>), g, b, 0, s, L, y, o);
    else hipLaunchKernelGGL((k_measure4<T, 8, 16, 0>), g, b, 0, s, L, y, o);
    return;
  }
  VP_DISPATCH_DC(k_measure4, T, L, y, o);
}
// One persistent launch: `grid` work-groups drain the item queue.
template <typename T>
void launch_sweep_queue(const LatDev& L0, const LatDev* lats, const SampleOut* outs, int measure, const int2* items,
                        int n_items, int* next, bool bf16, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, next);
  const LatDev& L = L0;
#define VP_SQ(DD, CC, BF)                                                                              \
  hipLaunchKernelGGL((k_sweep_queue<T, DD, CC, BF>), dim3(grid), dim3(WG), 0, s, lats, outs, measure, items, \
                     n_items, next)
#define VP_SQ_SHAPE(BF)                                                                                \
  do {                                                                                                 \
    if (L.d == 8 && L.c == 16) VP_SQ(8, 16, BF);                                                       \
    else if (L.d == 6 && L.c == 12) VP_SQ(6, 12, BF);                                                  \
    else if (L.d == 4 && L.c == 8) VP_SQ(4, 8, BF);                                                    \
    else VP_SQ(0, 0, BF);                                                                              \
  } while (0)
  if constexpr (sizeof(T) == 8) {
    if (bf16) {
      VP_SQ_SHAPE(true);
      return;
    }
  }
  VP_SQ_SHAPE(false);
#undef VP_SQ_SHAPE
#undef VP_SQ
}

// Work-groups of the persistent kernel that fit on one CU at once.
template <typename T>
int sweep_queue_occupancy(const LatDev& L, bool bf16) {
  int n = 0;
#define VP_OCC(DD, CC, BF) hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_sweep_queue<T, DD, CC, BF>, WG, 0)
  auto shape = [&](auto bf) {
    constexpr bool BF = decltype(bf)::value;
    if (L.d == 8 && L.c == 16) VP_OCC(8, 16, BF);
    else if (L.d == 6 && L.c == 12) VP_OCC(6, 12, BF);
    else if (L.d == 4 && L.c == 8) VP_OCC(4, 8, BF);
    else VP_OCC(0, 0, BF);
  };
  if constexpr (sizeof(T) == 8) {
    if (bf16) shape(std::true_type{});
    else shape(std::false_type{});
  } else {
    shape(std::false_type{});
  }
#undef VP_OCC
  return n;
}

// The library compiles this file once per working type (VP_KERNEL_UNIT 0:
// float64 and the type-independent launchers, 1: float32) so that the two
// halves build side by side.
#if VP_KERNEL_UNIT == 0
void launch_begin_sample(const LatDev& L, hipStream_t s) {
  hipLaunchKernelGGL(k_begin_sample, dim3((L.n_chains + WG - 1) / WG), dim3(WG), 0, s, L);
}
void launch_finish_sample(const LatDev& L, const SampleOut& o, int n_active, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_sample, dim3(n_active), dim3(64), 0, s, L, o, n_active);
}
void launch_next_sweep(const LatDev& L, hipStream_t s) {
  hipLaunchKernelGGL(k_next_sweep, dim3((L.n_chains + WG - 1) / WG), dim3(WG), 0, s, L);
}
void launch_init_tensors(double* T, int64_t Np, uint64_t seed, int lat_id, double scale, double perturb,
                         hipStream_t s) {
  int blocks = (int)std::min<int64_t>((Np + WG - 1) / WG, 65536);
  hipLaunchKernelGGL(k_init_tensors, dim3(blocks), dim3(WG), 0, s, T, Np, seed, lat_id, scale, perturb);
}
void launch_init_chains(const LatDev& L, hipStream_t s) {
  hipLaunchKernelGGL(k_init_chains, dim3((L.n_chains + 63) / 64), dim3(64), 0, s, L);
}
void launch_copy_spins(const LatDev& L, const int8_t* src, int n_cfg, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_spins, dim3(n_cfg), dim3(64), 0, s, L, src, n_cfg);
}
#endif
template <typename T>
void launch_gradient(const int64_t* offs, const int64_t* coff, const int32_t* sz, int N, int64_t Np,
                     const double* e, const T* dl, const int8_t* spins, int64_t ns, double* grad, double* emean,
                     double* work, hipStream_t s) {
  (void)work;
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(WG), 0, s, e, ns, emean);
  int64_t nh = Np / 2;
  hipLaunchKernelGGL(k_gradient<T>, dim3((unsigned)((nh + WG - 1) / WG)), dim3(WG), 0, s, offs, coff, sz, N, e, dl,
                     spins, ns, nh, (const double*)emean, grad);
}
#if VP_KERNEL_UNIT == 0
void launch_sign_sgd(double* T, const double* g, int64_t Np, double step_len, uint64_t seed, int lat_id,
                     uint64_t step, hipStream_t s) {
  int blocks = (int)std::min<int64_t>((Np + WG - 1) / WG, 65536);
  hipLaunchKernelGGL(k_sign_sgd, dim3(blocks), dim3(WG), 0, s, T, g, Np, step_len, seed, lat_id, step);
}
#endif

#define VP_INSTANTIATE(T)                                                                            \
  template void launch_prepare_tensors<T>(const LatDev&, const double*, T*, const int64_t*, hipStream_t); \
  template void launch_init_trivial<T>(const LatDev&, hipStream_t);                                  \
  template void launch_row3_right<T>(const LatDev&, int, int, int, bool, hipStream_t);                    \
  template void launch_hsweep<T>(const LatDev&, int, int, bool, hipStream_t);                             \
  template void launch_psi_fixed<T>(const LatDev&, hipStream_t);                                    \
  template void launch_row4_right<T>(const LatDev&, int, bool, hipStream_t);                              \
  template void launch_vsweep<T>(const LatDev&, int, bool, bool, hipStream_t);                                \
  template void launch_hsweep_pair<T>(const LatDev&, int, int, bool, hipStream_t);                            \
  template void launch_vsweep_pair<T>(const LatDev&, int, bool, hipStream_t);                                 \
  template void launch_sweep_queue<T>(const LatDev&, const LatDev*, const SampleOut*, int, const int2*, int, int*, \
                                      bool, int, hipStream_t);                                              \
  template int sweep_queue_occupancy<T>(const LatDev&, bool);                                \
  template void launch_compress<T>(const LatDev&, int, int, hipStream_t);                           \
  template void launch_measure3<T>(const LatDev&, int, const SampleOut&, hipStream_t);              \
  template void launch_measure4<T>(const LatDev&, int, const SampleOut&, hipStream_t);              \
  template void launch_gradient<T>(const int64_t*, const int64_t*, const int32_t*, int, int64_t,    \
                                   const double*, const T*, const int8_t*, int64_t, double*, double*, \
                                   double*, hipStream_t);

#if VP_KERNEL_UNIT == 0
VP_INSTANTIATE(double)
#else
VP_INSTANTIATE(float)
#endif

}  // namespace vp
