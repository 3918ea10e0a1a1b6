// Host runtime and C ABI of the VMC-PEPS library: context and workspace
// planning, tensor staging, and the sweep schedule that enqueues the phase
// kernels row by row on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vmcpeps.h"
#include "vp_kernels.hpp"
#include "vp_net.hpp"

using namespace vp;

namespace {

// A transposed lattice kept beside a caller's lattice (site (y,x) -> (x,y), the
// same state): TWIN_COLUMNS carries the vertical bonds of VP_VERT_COLUMN as its
// horizontal ones; TWIN_KNIGHTS evaluates the triangular lattice's knight bonds
// (y,x)-(y+2,x+1) as its own (x,y)-(x+1,y+2) ones.
enum { TWIN_NONE = 0, TWIN_COLUMNS = 1, TWIN_KNIGHTS = 2 };

struct Lattice {
  vp_lattice p{};
  int N = 0;
  int64_t Np = 0;
  std::vector<int64_t> offs;    // canonical offsets per site (N+1)
  std::vector<int64_t> coff;    // compact offsets per site (N+1)
  std::vector<int32_t> dims;    // [N][4]
  std::vector<int32_t> sizes;   // l*u*r*d per site
  std::vector<int32_t> kU, kD;  // boundary bond dims
  size_t tsize = 8;             // bytes of the working type
  // device buffers
  double* T = nullptr;          // canonical float64 tensors
  void* Tw = nullptr;           // padded working tensors
  void* ws = nullptr;
  double* cws = nullptr;
  int32_t* iws = nullptr;
  double* dws = nullptr;
  ChainMeta* meta = nullptr;
  int8_t* spins = nullptr;
  int32_t *d_kU = nullptr, *d_kD = nullptr, *d_dims = nullptr, *d_sizes = nullptr;
  int64_t *d_offs = nullptr, *d_coff = nullptr;
  double* d_scratch = nullptr;  // small scalar scratch
  // proposal network: float32 master, working-precision copy, Adam moments
  float* d_net = nullptr;
  double* d_net64 = nullptr;
  char* d_netbf = nullptr;      // packed bf16 copy (bf16 inference in the bf16 sampling mode)
  float* d_adam = nullptr;      // [2][NET_NPARAM]: m, v
  int64_t adam_t = 0;
  bool net_ready = false;
  int32_t sampler = VP_SAMPLER_PAIR_SEQ;
  int32_t schedule = VP_SCHED_PHASES;
  int64_t sweeps = 0;           // sweeps since vp_init_chains (every chain's counter)
  // spin-inversion scratch, reserved at vp_create: reversed configurations
  // [n_chains][N], then log|Psi(Sbar)|, E_loc(Sbar) [n_chains] and sign(Sbar)
  char* d_sis = nullptr;
  // workspaces whose size depends on call arguments (SR, optimisation loop,
  // proposal network): allocated on first use, grown when a later call needs
  // more, released by vp_destroy
  struct Buf {
    void* p = nullptr;
    size_t cap = 0;
  };
  Buf sr_work, sr_flag, opt_lp, opt_el, opt_grad, opt_em, opt_sg, opt_so, opt_dl;
  Buf nw_work, nw_part, nw_cnt, nw_scal, nw_grad, nw_sb, nw_rb, nw_idx;
  // simple update: site tensors, link lambdas, per-link changes, per-work-group scratch
  Buf su_B, su_lam, su_change, su_scr;
  // VP_VERT_COLUMN evaluation: the transposed lattice's pair ratios
  Buf col_ratios;
  bool su_valid = false;        // su_B / su_lam hold the evolution of the current tensors
  LatDev dev{};
  bool tensors_ready = false;
  bool chains_ready = false;
  bool lower_valid = false;     // D boundaries match the current spins
  int col = -1;                 // index of the transposed lattice in vp_ctx::lats, else -1
  int role = 0;                 // what that lattice does: TWIN_COLUMNS or TWIN_KNIGHTS
};

}  // namespace

struct vp_ctx {
  std::vector<Lattice> lats;         // the caller's lattices, then the transposed ones of VP_VERT_COLUMN
  int32_t n_user = 0;                // lattices the caller indexes
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  std::string err;
  // phase timing
  bool timing = false;
  std::vector<hipEvent_t> ev;        // pairs: start, stop
  std::vector<int> ev_phase;
  size_t ev_used = 0;
  double ph_ms[VP_NPHASE] = {0};
  int64_t ph_n[VP_NPHASE] = {0};
  // persistent-launch tables (device) and their host images
  LatDev* q_lats = nullptr;
  SampleOut* q_outs = nullptr;
  int2* q_items = nullptr;
  int* q_next = nullptr;
  size_t q_lat_cap = 0, q_item_cap = 0;
  std::vector<LatDev> h_lats;
  std::vector<SampleOut> h_outs;
  std::vector<int2> h_items;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  hipEvent_t cap_event = nullptr;
};

namespace {

thread_local std::string g_err;

vp_status fail(vp_ctx* ctx, vp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  g_err = buf;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail((ctx), VP_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Makes b hold at least `bytes`; a larger buffer replaces it once the stream has
// finished with the old one.
bool grow(hipStream_t s, Lattice::Buf& b, size_t bytes) {
  if (b.p && b.cap >= bytes) return true;
  if (b.p) {
    hipStreamSynchronize(s);
    hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  if (hipMalloc(&b.p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    b.p = nullptr;
    return false;
  }
  b.cap = std::max<size_t>(bytes, 256);
  return true;
}

size_t sis_bytes(const vp_lattice& p) {
  const size_t nb = (size_t)p.n_chains * p.Ly * p.Lx;
  return (nb + 255) / 256 * 256 + 2 * sizeof(double) * p.n_chains + p.n_chains;
}

void site_dims(const vp_lattice& p, int y, int x, int32_t out[4]) {
  out[0] = x > 0 ? p.D : 1;
  out[1] = y > 0 ? p.D : 1;
  out[2] = x < p.Lx - 1 ? p.D : 1;
  out[3] = y < p.Ly - 1 ? p.D : 1;
}

// Bond dimensions of every boundary MPS produced by the canonical compression:
// alpha'_0 = 1, alpha'_{j+1} = min(alpha'_j p_j, alpha_{j+1}); k_j = min(Dc, alpha'_j, p_j k_{j+1}).
void plan_bonds(Lattice& L) {
  const vp_lattice& p = L.p;
  const int W = p.Lx + 1;
  L.kU.assign((size_t)(p.Ly + 1) * W, 1);
  L.kD.assign((size_t)(p.Ly + 1) * W, 1);
  auto compress_dims = [&](const int32_t* kin, int y, bool upper, int32_t* kout) {
    std::vector<int64_t> alpha(W), ap(W);
    for (int j = 0; j <= p.Lx; ++j) {
      int l = (j == 0 || j == p.Lx) ? 1 : p.D;
      alpha[j] = (int64_t)kin[j] * l;
    }
    auto phys = [&](int j) {
      int32_t dd[4];
      site_dims(p, y, j, dd);
      return upper ? dd[3] : dd[1];
    };
    ap[0] = 1;
    for (int j = 0; j < p.Lx; ++j) ap[j + 1] = std::min<int64_t>(ap[j] * phys(j), alpha[j + 1]);
    kout[p.Lx] = 1;
    for (int j = p.Lx - 1; j >= 1; --j)
      kout[j] = (int32_t)std::min<int64_t>(std::min<int64_t>(p.Dc, ap[j]), (int64_t)phys(j) * kout[j + 1]);
    kout[0] = 1;
  };
  for (int y = 0; y <= p.Ly - 2; ++y) compress_dims(&L.kU[(size_t)y * W], y, true, &L.kU[(size_t)(y + 1) * W]);
  for (int y = p.Ly - 1; y >= 1; --y) compress_dims(&L.kD[(size_t)(y + 1) * W], y, false, &L.kD[(size_t)y * W]);
}

struct Plan {
  int64_t ws = 0, iws = 0, dws = 0, cws = 0;
};

Plan plan_workspace(const vp_lattice& p, LatDev* dev) {
  const int64_t c = p.Dc, d = p.D, Lx = p.Lx, Ly = p.Ly;
  const int64_t s3 = c * d * c, s4 = c * d * d * c, sx = c * c * d * d * d;
  int64_t o = 0;
  auto take = [&](int64_t n) {
    int64_t r = o;
    o += (n + 63) & ~int64_t(63);
    return r;
  };
  LatDev L{};
  L.oUb = take((Ly + 1) * Lx * s3);
  L.oDb = take((Ly + 1) * Lx * s3);
  L.oL3 = take((Lx + 1) * s3);
  L.oR3 = take((Lx + 1) * s3);
  L.oT3 = take(4 * s3);
  L.oL4 = take((Lx + 1) * s4);
  L.oR4 = take((Lx + 1) * s4);
  L.oT4 = take(4 * s4);
  L.oX0 = take(sx);
  L.oX1 = take(sx);
  L.oDl = take(d * d * d * d);
  Plan P;
  P.ws = o;
  o = 0;
  L.cG = take(Lx * s4);
  L.cX0 = take(sx);
  L.cX1 = take(sx);
  L.cY = take(s4);
  L.cW = take(s4);
  L.cH = take(s4);
  L.cHc = take(s4);
  L.cVk = take(s4);
  L.cVp = take(s3);
  L.cTa = take(s3);
  L.cTb = take(s3);
  L.cRefl = take(128 * 129 / 2);
  L.cLam = take(64);
  P.cws = o;
  int64_t io = 0;
  L.ieL3 = io; io += Lx + 2;
  L.ieR3 = io; io += Lx + 2;
  L.ieT3 = io; io += 4;
  L.ieL4 = io; io += Lx + 2;
  L.ieR4 = io; io += Lx + 2;
  L.ieT4 = io; io += 4;
  P.iws = (io + 15) & ~int64_t(15);
  L.dlamU = 0;
  L.dlamD = Ly + 1;
  P.dws = ((2 * (Ly + 1)) + 7) & ~int64_t(7);
  if (dev) *dev = L;
  return P;
}

// Working precision: float32 for VP_FP32; float64 for VP_FP64 and VP_BF16 (whose
// bf16 operands are rounded from float64 storage inside the sampling kernels).
bool works_f64(int prec) { return prec != VP_FP32; }
size_t type_size(int prec) { return works_f64(prec) ? 8 : 4; }

vp_status check_lattice(vp_ctx* ctx, const vp_lattice& p) {
  if (p.Ly < 1 || p.Lx < 1 || p.D < 1 || p.Dc < 1 || p.n_chains < 1)
    return fail(ctx, VP_ERR_SHAPE, "Ly, Lx, D, Dc and n_chains must be >= 1");
  if ((p.Ly * p.Lx) % 2)
    return fail(ctx, VP_ERR_SHAPE, "the S^z_tot = 0 sector needs an even number of sites");
  if (p.Ly * p.Lx > 4096) return fail(ctx, VP_ERR_SHAPE, "at most 4096 sites");
  if (p.prec != VP_FP64 && p.prec != VP_FP32 && p.prec != VP_BF16)
    return fail(ctx, VP_ERR_ARG, "unknown precision %d", p.prec);
  if (p.compress != VP_COMPRESS_CANONICAL && p.compress != VP_COMPRESS_VARIATIONAL)
    return fail(ctx, VP_ERR_ARG, "unknown truncation mode %d", p.compress);
  // the canonical compression's eigenproblems have order up to D*Dc (at most
  // 128 in registers); the fit has none, and its QRs take up to 64 columns
  if (p.D > 16 || p.Dc > 64) return fail(ctx, VP_ERR_SHAPE, "sizes beyond the built kernels (D <= 16, Dc <= 64)");
  if (p.compress == VP_COMPRESS_CANONICAL && p.D * p.Dc > 128)
    return fail(ctx, VP_ERR_SHAPE, "the canonical compression needs D*Dc <= 128");
  if (p.compress == VP_COMPRESS_VARIATIONAL && p.D * p.Dc > 192)
    return fail(ctx, VP_ERR_SHAPE, "the variational fit needs D*Dc <= 192");
  if (p.fit_sweeps < 0 || p.fit_sweeps > 64) return fail(ctx, VP_ERR_ARG, "fit_sweeps must be 0..64");
  if (p.geometry != VP_GEOM_SQUARE && p.geometry != VP_GEOM_TRIANGULAR)
    return fail(ctx, VP_ERR_ARG, "unknown geometry %d", p.geometry);
  if (p.vertical != VP_VERT_ROWPAIR && p.vertical != VP_VERT_COLUMN)
    return fail(ctx, VP_ERR_ARG, "unknown vertical-bond mode %d", p.vertical);
  if (p.vertical == VP_VERT_COLUMN && (p.J2 != 0.0 || p.geometry != VP_GEOM_SQUARE))
    return fail(ctx, VP_ERR_UNSUPPORTED, "column-wise vertical bonds: nearest-neighbour square lattices only");
  return VP_OK;
}

// The transposed lattice of a VP_VERT_COLUMN lattice: Lx x Ly, everything else equal.
vp_lattice transposed_params(const vp_lattice& p) {
  vp_lattice t = p;
  t.Ly = p.Lx;
  t.Lx = p.Ly;
  t.vertical = VP_VERT_ROWPAIR;
  return t;
}

// Couplings of the diagonal (y,x)-(y+1,x+1) and the anti-diagonal (y,x+1)-(y+1,x).
double diag_coupling(const vp_lattice& p) { return p.geometry == VP_GEOM_TRIANGULAR ? p.J1 : p.J2; }
double anti_coupling(const vp_lattice& p) { return p.J2; }
bool has_diagonals(const vp_lattice& p) { return diag_coupling(p) != 0.0 || anti_coupling(p) != 0.0; }
// The triangular lattice's knight bonds (y,x)-(y+1,x+2) and (y,x)-(y+2,x+1), coupling J2.
bool has_knights(const vp_lattice& p) { return p.geometry == VP_GEOM_TRIANGULAR && p.J2 != 0.0; }
// Pairs of the ratio outputs: horizontal, vertical, two diagonals per plaquette, knight bonds.
int n_pairs_of(const vp_lattice& p) {
  int n = p.Ly * (p.Lx - 1) + (p.Ly - 1) * p.Lx;
  if (has_diagonals(p)) n += 2 * (p.Ly - 1) * (p.Lx - 1);
  if (has_knights(p)) n += (p.Ly - 1) * std::max(p.Lx - 2, 0) + std::max(p.Ly - 2, 0) * (p.Lx - 1);
  return n;
}

Lattice* get_lat(vp_ctx* ctx, int32_t lat) {
  if (!ctx || lat < 0 || lat >= ctx->n_user) return nullptr;
  return &ctx->lats[lat];
}

// Brackets phase launches with HIP events while timing is enabled.
struct Rec {
  vp_ctx* ctx;
  int phase = -1;
  explicit Rec(vp_ctx* c) : ctx(c) {}
  void begin(int ph) {
    if (!ctx->timing) return;
    if (ctx->ev_used + 2 > ctx->ev.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { ctx->timing = false; return; }
        ctx->ev.push_back(e);
      }
      ctx->ev_phase.resize(ctx->ev.size() / 2);
    }
    phase = ph;
    hipEventRecord(ctx->ev[ctx->ev_used], ctx->stream);
  }
  void end() {
    if (!ctx->timing || phase < 0) return;
    hipEventRecord(ctx->ev[ctx->ev_used + 1], ctx->stream);
    ctx->ev_phase[ctx->ev_used / 2] = phase;
    ctx->ev_used += 2;
    phase = -1;
  }
};

void fold_timing(vp_ctx* ctx) {
  if (ctx->ev_used == 0) return;
  hipStreamSynchronize(ctx->stream);
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]) == hipSuccess) {
      ctx->ph_ms[ctx->ev_phase[i / 2]] += ms;
      ctx->ph_n[ctx->ev_phase[i / 2]] += 1;
    }
  }
  ctx->ev_used = 0;
}

#define TIMED(rec, ph, call) \
  do {                       \
    (rec).begin(ph);         \
    call;                    \
    (rec).end();             \
  } while (0)

template <typename T>
void run_lower_pass(vp_ctx* ctx, Lattice& L, hipStream_t s) {
  Rec r(ctx);
  for (int y = L.p.Ly - 1; y >= 1; --y) TIMED(r, VP_PH_COMPRESS_DOWN, launch_compress<T>(L.dev, y, 0, s));
}

template <typename T>
void run_sweep(vp_ctx* ctx, Lattice& L, const SampleOut* o, hipStream_t s) {
  const int Ly = L.p.Ly;
  // VP_BF16: the sampling pass contracts with bf16 operands (f32 accumulation);
  // measurement and compression run in float64.
  const bool bf = L.p.prec == VP_BF16;
  Rec r(ctx);
  // top-down sampling pass
  for (int y = 0; y < Ly; ++y) {
    TIMED(r, VP_PH_ROW3_ENVS, launch_row3_right<T>(L.dev, y, y, y + 1, bf, s));
    TIMED(r, VP_PH_HSWEEP, launch_hsweep<T>(L.dev, y, y == Ly - 1, bf, s));
    if (y < Ly - 1) {
      TIMED(r, VP_PH_ROW4_ENVS, launch_row4_right<T>(L.dev, y, bf, s));
      TIMED(r, VP_PH_VSWEEP, launch_vsweep<T>(L.dev, y, bf, L.sampler == VP_SAMPLER_LEARNED_PLAQ, s));
      TIMED(r, VP_PH_COMPRESS_UP, launch_compress<T>(L.dev, y, 1, s));
    }
  }
  // bottom-up measurement pass, rebuilding the lower boundaries
  if (o) TIMED(r, VP_PH_OTHER, launch_begin_sample(L.dev, s));
  for (int y = Ly - 1; y >= 0; --y) {
    if (o) {
      TIMED(r, VP_PH_MEASURE3, launch_measure3<T>(L.dev, y, *o, s));
      if (y < Ly - 1) TIMED(r, VP_PH_MEASURE4, launch_measure4<T>(L.dev, y, *o, s));
    }
    if (y >= 1) TIMED(r, VP_PH_COMPRESS_DOWN, launch_compress<T>(L.dev, y, 0, s));
  }
  if (o) TIMED(r, VP_PH_OTHER, launch_finish_sample(L.dev, *o, L.p.n_chains, s));
  TIMED(r, VP_PH_OTHER, launch_next_sweep(L.dev, s));
  if (ctx->ev_used >= 8192) fold_timing(ctx);
}

// Persistent schedule: every chain of every lattice in one launch per sweep.
// All lattices share d, c and the working precision.
template <typename T>
vp_status run_queue(vp_ctx* ctx, const std::vector<Lattice*>& lats, int n_burn, int n_meas,
                    const std::vector<SampleOut>& outs, hipStream_t s) {
  const int n = (int)lats.size();
  for (const Lattice* L : lats)
    if (L->p.compress != VP_COMPRESS_CANONICAL)
      return fail(ctx, VP_ERR_UNSUPPORTED, "the persistent schedule runs the canonical compression only");
  // the tables are rewritten: the previous call's launches must be done
  HIP_TRY(ctx, hipStreamSynchronize(s));
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lats[a]->N > lats[b]->N; });
  ctx->h_lats.resize(n);
  ctx->h_outs.assign(outs.begin(), outs.end());
  ctx->h_items.clear();
  for (int i = 0; i < n; ++i) {
    ctx->h_lats[i] = lats[i]->dev;
    ctx->h_lats[i].learned = lats[i]->sampler == VP_SAMPLER_LEARNED_PLAQ;
  }
  // largest lattices first: their sweeps start early and the short ones fill the tail
  for (int i : order)
    for (int ch = 0; ch < lats[i]->p.n_chains; ++ch) ctx->h_items.push_back(int2{i, ch});
  const size_t ni = ctx->h_items.size();
  if (ctx->q_lat_cap < (size_t)n) {
    if (ctx->q_lats) hipFree(ctx->q_lats);
    if (ctx->q_outs) hipFree(ctx->q_outs);
    ctx->q_lats = nullptr; ctx->q_outs = nullptr;
    if (hipMalloc((void**)&ctx->q_lats, sizeof(LatDev) * n) != hipSuccess ||
        hipMalloc((void**)&ctx->q_outs, sizeof(SampleOut) * n) != hipSuccess)
      return fail(ctx, VP_ERR_OOM, "persistent-launch tables");
    ctx->q_lat_cap = n;
  }
  if (ctx->q_item_cap < ni) {
    if (ctx->q_items) hipFree(ctx->q_items);
    ctx->q_items = nullptr;
    if (hipMalloc((void**)&ctx->q_items, sizeof(int2) * ni) != hipSuccess)
      return fail(ctx, VP_ERR_OOM, "persistent-launch work list");
    ctx->q_item_cap = ni;
  }
  if (!ctx->q_next && hipMalloc((void**)&ctx->q_next, sizeof(int)) != hipSuccess)
    return fail(ctx, VP_ERR_OOM, "persistent-launch counter");
  HIP_TRY(ctx, hipMemcpyAsync(ctx->q_lats, ctx->h_lats.data(), sizeof(LatDev) * n, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->q_outs, ctx->h_outs.data(), sizeof(SampleOut) * n, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->q_items, ctx->h_items.data(), sizeof(int2) * ni, hipMemcpyHostToDevice, s));
  const bool bf = lats[0]->p.prec == VP_BF16;
  int dev = 0, cus = 0;
  HIP_TRY(ctx, hipGetDevice(&dev));
  HIP_TRY(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int occ = std::max(1, sweep_queue_occupancy<T>(lats[0]->dev, bf));
  const int grid = (int)std::min<size_t>(ni, (size_t)cus * occ);
  Rec r(ctx);
  for (int i = 0; i < n_burn + n_meas; ++i) {
    TIMED(r, VP_PH_OTHER, launch_sweep_queue<T>(lats[0]->dev, ctx->q_lats, ctx->q_outs, i >= n_burn ? 1 : 0,
                                                 ctx->q_items, (int)ni, ctx->q_next, bf, grid, s));
    HIP_TRY(ctx, hipGetLastError());
  }
  if (ctx->ev_used >= 8192) fold_timing(ctx);
  return VP_OK;
}

// Graph schedule: the per-phase launches of one sweep captured once per call
// (one graph without and one with measurement) and replayed every sweep.
template <typename T>
vp_status run_graph(vp_ctx* ctx, Lattice& L, int n_burn, int n_meas, const SampleOut& o, hipStream_t s) {
  if (!ctx->cap_stream) {
    HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->cap_event, hipEventDisableTiming));
  }
  if (ctx->ev_used) fold_timing(ctx);  // no event synchronisation may happen while capturing
  const bool timing = ctx->timing;
  ctx->timing = false;  // no event records inside the graphs
  hipGraph_t g[2] = {nullptr, nullptr};
  hipGraphExec_t x[2] = {nullptr, nullptr};
  vp_status st = VP_OK;
  for (int k = 0; k < 2 && st == VP_OK; ++k) {
    if ((k == 0 && n_burn == 0) || (k == 1 && n_meas == 0)) continue;
    if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = fail(ctx, VP_ERR_DEVICE, "graph capture could not begin");
      break;
    }
    run_sweep<T>(ctx, L, k == 1 ? &o : nullptr, ctx->cap_stream);
    if (hipStreamEndCapture(ctx->cap_stream, &g[k]) != hipSuccess ||
        hipGraphInstantiate(&x[k], g[k], nullptr, nullptr, 0) != hipSuccess)
      st = fail(ctx, VP_ERR_DEVICE, "graph capture of the sweep failed");
  }
  ctx->timing = timing;
  Rec r(ctx);
  for (int i = 0; i < n_burn + n_meas && st == VP_OK; ++i) {
    TIMED(r, VP_PH_OTHER, hipGraphLaunch(x[i >= n_burn ? 1 : 0], s));
    if (hipGetLastError() != hipSuccess) st = fail(ctx, VP_ERR_DEVICE, "graph launch failed");
  }
  // the executable graphs are released once their launches are done
  hipStreamSynchronize(s);
  for (int k = 0; k < 2; ++k) {
    if (x[k]) hipGraphExecDestroy(x[k]);
    if (g[k]) hipGraphDestroy(g[k]);
  }
  return st;
}

template <typename T>
void run_eval(const LatDev& D, const SampleOut& o, int n_cfg, hipStream_t s, bool rowpair = true, bool rows = true) {
  const int Ly = D.Ly;
  for (int y = 0; y < Ly - 1; ++y) launch_compress<T>(D, y, 1, s);
  launch_psi_fixed<T>(D, s);
  launch_begin_sample(D, s);
  for (int y = Ly - 1; y >= 0; --y) {
    if (rows) launch_measure3<T>(D, y, o, s);
    if (y < Ly - 1 && rowpair) launch_measure4<T>(D, y, o, s);
    if (y >= 1) launch_compress<T>(D, y, 0, s);
  }
  launch_finish_sample(D, o, n_cfg, s);
}

// Per-chain scratch of one measurement (log|Psi|, E_loc, sign), in the region
// reserved at vp_create after the spin-inversion configurations.
SampleOut scratch_out(Lattice& L) {
  const size_t nb = (size_t)L.p.n_chains * L.N;
  const size_t off_l = (nb + 255) / 256 * 256, off_e = off_l + sizeof(double) * L.p.n_chains,
               off_s = off_e + sizeof(double) * L.p.n_chains;
  SampleOut o{};
  o.log_abs_psi = (double*)(L.d_sis + off_l);
  o.e_loc = (double*)(L.d_sis + off_e);
  o.sign = (int8_t*)(L.d_sis + off_s);
  o.n_meas = 1;
  o.m = 0;
  o.dyn_m = 0;
  o.np_half = L.Np / 2;
  return o;
}

// TWIN_KNIGHTS: the knight bonds (y,x)-(y+2,x+1) of the n configurations in L's
// chain slots, evaluated as the transposed lattice's (x,y)-(x+1,y+2) bonds (its
// 2-row measurement with every other term switched off); their energies are
// added into row m of e ([n][n_meas]) and, when r is given, their ratios placed
// in r ([n][np]) after the pairs the 2-row measurement writes.
template <typename T>
bool eval_knights(vp_ctx* ctx, Lattice& L, int n, double* e, int n_meas, int m, double* r, int np, hipStream_t s) {
  Lattice& C = ctx->lats[L.col];
  const vp_lattice& p = L.p;
  launch_transpose_spins(L.spins, (int8_t*)C.d_sis, n, p.Ly, p.Lx, true, s);
  launch_copy_spins(C.dev, (const int8_t*)C.d_sis, n, s);  // clears the transposed chains' flags
  LatDev Dt = C.dev;
  Dt.n_chains = n;
  SampleOut oc = scratch_out(C);
  // the transposed lattice's ratio layout: its nearest-neighbour pairs, then its knight bonds
  const int base_t = C.p.Ly * (C.p.Lx - 1) + (C.p.Ly - 1) * C.p.Lx;
  const int npt = base_t + (C.p.Ly - 1) * std::max(C.p.Lx - 2, 0);
  oc.n_pairs = npt;
  if (r) {
    if (!grow(s, C.col_ratios, sizeof(double) * (size_t)n * npt)) return false;
    oc.ratios = (double*)C.col_ratios.p;
  }
  run_eval<T>(Dt, oc, n, s, true, false);
  launch_add_energy(e, n_meas, m, oc.e_loc, n, s);
  if (r) {
    const int base_r = np - std::max(p.Ly - 2, 0) * (p.Lx - 1);
    launch_knight_ratios(oc.ratios, npt, base_t, r, np, base_r, n, p.Ly, p.Lx, s);
  }
  return true;
}

// VP_VERT_COLUMN sampling: every sweep visits the horizontal bonds with the row
// boundaries, then the vertical bonds as the horizontal bonds of the transposed
// lattice C (after its own lower-boundary pass); a measured sweep evaluates the
// final configuration: the rows' upper boundaries afresh and their measurement
// pass (Psi, horizontal terms, G), then C's measurement pass (its upper
// boundaries are those of its pass), whose energies are added to the rows'.
template <typename T>
vp_status run_col_sample(vp_ctx* ctx, Lattice& L, Lattice& C, int n_burn, int n_meas, SampleOut o) {
  hipStream_t s = ctx->stream;
  const int Ly = L.p.Ly, Lx = L.p.Lx, n = L.p.n_chains;
  const bool bf = L.p.prec == VP_BF16;
  if (!L.lower_valid) {
    run_lower_pass<T>(ctx, L, s);
    L.lower_valid = true;
  }
  o.psi_meas = 1;  // Psi of the final configuration, from the rows' measurement pass
  SampleOut oc = scratch_out(C);
  oc.psi_meas = 0;
  Rec r(ctx);
  for (int i = 0; i < n_burn + n_meas; ++i) {
    for (int y = 0; y < Ly; ++y) {
      TIMED(r, VP_PH_ROW3_ENVS, launch_row3_right<T>(L.dev, y, y, y + 1, bf, s));
      TIMED(r, VP_PH_HSWEEP, launch_hsweep<T>(L.dev, y, y == Ly - 1, bf, s));
      if (y < Ly - 1) TIMED(r, VP_PH_COMPRESS_UP, launch_compress<T>(L.dev, y, 1, s));
    }
    launch_transpose_spins(L.spins, C.spins, n, Ly, Lx, true, s);
    run_lower_pass<T>(ctx, C, s);
    for (int y = 0; y < Lx; ++y) {
      TIMED(r, VP_PH_ROW3_ENVS, launch_row3_right<T>(C.dev, y, y, y + 1, bf, s));
      TIMED(r, VP_PH_HSWEEP, launch_hsweep<T>(C.dev, y, y == Lx - 1, bf, s));
      if (y < Lx - 1) TIMED(r, VP_PH_COMPRESS_UP, launch_compress<T>(C.dev, y, 1, s));
    }
    launch_transpose_spins(C.spins, L.spins, n, Ly, Lx, false, s);
    if (i >= n_burn) {
      for (int y = 0; y < Ly - 1; ++y) TIMED(r, VP_PH_COMPRESS_UP, launch_compress<T>(L.dev, y, 1, s));
      TIMED(r, VP_PH_OTHER, launch_begin_sample(L.dev, s));
      for (int y = Ly - 1; y >= 0; --y) {
        TIMED(r, VP_PH_MEASURE3, launch_measure3<T>(L.dev, y, o, s));
        if (y >= 1) TIMED(r, VP_PH_COMPRESS_DOWN, launch_compress<T>(L.dev, y, 0, s));
      }
      TIMED(r, VP_PH_OTHER, launch_finish_sample(L.dev, o, n, s));
      TIMED(r, VP_PH_OTHER, launch_begin_sample(C.dev, s));
      for (int y = Lx - 1; y >= 0; --y) {
        TIMED(r, VP_PH_MEASURE3, launch_measure3<T>(C.dev, y, oc, s));
        if (y >= 1) TIMED(r, VP_PH_COMPRESS_DOWN, launch_compress<T>(C.dev, y, 0, s));
      }
      TIMED(r, VP_PH_OTHER, launch_finish_sample(C.dev, oc, n, s));
      launch_add_energy(o.e_loc, n_meas, i - n_burn, oc.e_loc, n, s);
    } else {
      for (int y = Ly - 1; y >= 1; --y) TIMED(r, VP_PH_COMPRESS_DOWN, launch_compress<T>(L.dev, y, 0, s));
    }
    TIMED(r, VP_PH_OTHER, launch_next_sweep(L.dev, s));
    TIMED(r, VP_PH_OTHER, launch_next_sweep(C.dev, s));
    HIP_TRY(ctx, hipGetLastError());
    if (ctx->ev_used >= 8192) fold_timing(ctx);
  }
  return VP_OK;
}

// Chains of |Phi|^2 (VP_SAMPLER_SIS_PAIR): chain c and c + n/2 carry S and its
// reversal.  Per call: the second half set to the reversal of the first, the
// lower boundaries and both top-down amplitudes contracted; then every sweep
// runs the plain phases over all chains and the decision phases over the pairs,
// and a measured sweep combines the two chains' measurements (taken into the
// scratch reserved at vp_create) into row m of the caller's outputs.
template <typename T>
vp_status run_pair_sample(vp_ctx* ctx, Lattice& L, int n_burn, int n_meas, double* log_abs_phi, int8_t* sign_phi,
                          double* e_loc_phi, int8_t* spins_out) {
  hipStream_t s = ctx->stream;
  const int Ly = L.p.Ly, n = L.p.n_chains, h = n / 2, N = L.N;
  const bool bf = L.p.prec == VP_BF16;
  launch_reverse_spins(L.spins, L.spins + (size_t)h * N, (int64_t)h * N, s);
  run_lower_pass<T>(ctx, L, s);
  L.lower_valid = true;
  for (int y = 0; y < Ly - 1; ++y) launch_compress<T>(L.dev, y, 1, s);
  launch_psi_fixed<T>(L.dev, s);
  HIP_TRY(ctx, hipGetLastError());
  // per-chain measurements of one sweep: log|Psi| [n], E_loc [n], sign [n]
  char* work = L.d_sis;
  const size_t nb = (size_t)n * N;
  const size_t off_l = (nb + 255) / 256 * 256, off_e = off_l + sizeof(double) * n, off_s = off_e + sizeof(double) * n;
  SampleOut o{};
  o.log_abs_psi = (double*)(work + off_l);
  o.e_loc = (double*)(work + off_e);
  o.sign = (int8_t*)(work + off_s);
  o.n_meas = 1;
  o.m = 0;
  o.dyn_m = 0;
  o.np_half = L.Np / 2;
  o.psi_meas = bf;
  Rec r(ctx);
  for (int i = 0; i < n_burn + n_meas; ++i) {
    const bool meas = i >= n_burn;
    for (int y = 0; y < Ly; ++y) {
      TIMED(r, VP_PH_ROW3_ENVS, launch_row3_right<T>(L.dev, y, y, y + 1, bf, s));
      TIMED(r, VP_PH_HSWEEP, launch_hsweep_pair<T>(L.dev, y, y == Ly - 1, bf, s));
      if (y < Ly - 1) {
        TIMED(r, VP_PH_ROW4_ENVS, launch_row4_right<T>(L.dev, y, bf, s));
        TIMED(r, VP_PH_VSWEEP, launch_vsweep_pair<T>(L.dev, y, bf, s));
        TIMED(r, VP_PH_COMPRESS_UP, launch_compress<T>(L.dev, y, 1, s));
      }
    }
    if (meas) TIMED(r, VP_PH_OTHER, launch_begin_sample(L.dev, s));
    for (int y = Ly - 1; y >= 0; --y) {
      if (meas) {
        TIMED(r, VP_PH_MEASURE3, launch_measure3<T>(L.dev, y, o, s));
        if (y < Ly - 1) TIMED(r, VP_PH_MEASURE4, launch_measure4<T>(L.dev, y, o, s));
      }
      if (y >= 1) TIMED(r, VP_PH_COMPRESS_DOWN, launch_compress<T>(L.dev, y, 0, s));
    }
    if (meas) {
      TIMED(r, VP_PH_OTHER, launch_finish_sample(L.dev, o, n, s));
      TIMED(r, VP_PH_OTHER, launch_pair_combine(h, n_meas, i - n_burn, o.log_abs_psi, o.sign, o.e_loc, L.spins, N,
                                                log_abs_phi, sign_phi, e_loc_phi, spins_out, s));
    }
    TIMED(r, VP_PH_OTHER, launch_next_sweep(L.dev, s));
    HIP_TRY(ctx, hipGetLastError());
    if (ctx->ev_used >= 8192) fold_timing(ctx);
  }
  return VP_OK;
}

vp_status check_flags(vp_ctx* ctx, Lattice& L) {
  std::vector<ChainMeta> m(L.p.n_chains), mc;
  HIP_TRY(ctx, hipMemcpyAsync(m.data(), L.meta, sizeof(ChainMeta) * m.size(), hipMemcpyDeviceToHost, ctx->stream));
  if (L.col >= 0) {  // the transposed lattice's chains
    mc.resize(m.size());
    HIP_TRY(ctx, hipMemcpyAsync(mc.data(), ctx->lats[L.col].meta, sizeof(ChainMeta) * mc.size(),
                                hipMemcpyDeviceToHost, ctx->stream));
  }
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (size_t i = 0; i < mc.size(); ++i) m[i].flags |= mc[i].flags;
  int zero = 0, nonfin = 0;
  for (auto& x : m) {
    zero += (x.flags & FLAG_ZERO) != 0;
    nonfin += (x.flags & FLAG_NONFINITE) != 0;
  }
  if (nonfin) return fail(ctx, VP_ERR_NONFINITE, "%d chain(s) produced a non-finite value", nonfin);
  if (zero) return fail(ctx, VP_ERR_ZERO_AMPLITUDE, "%d chain(s) met a zero amplitude", zero);
  return VP_OK;
}

// Checks that every configuration is 0/1 and in the S^z_tot = 0 sector.
vp_status check_configs(vp_ctx* ctx, const Lattice& L, const int8_t* spins_dev, int64_t n_cfg) {
  std::vector<int8_t> h((size_t)n_cfg * L.N);
  HIP_TRY(ctx, hipMemcpyAsync(h.data(), spins_dev, h.size(), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int64_t ch = 0; ch < n_cfg; ++ch) {
    int up = 0;
    for (int i = 0; i < L.N; ++i) {
      int8_t v = h[(size_t)ch * L.N + i];
      if (v != 0 && v != 1) return fail(ctx, VP_ERR_SHAPE, "spins must be 0 or 1");
      up += v;
    }
    if (2 * up != L.N)
      return fail(ctx, VP_ERR_SHAPE, "configuration %lld is not in the S^z_tot = 0 sector", (long long)ch);
  }
  return VP_OK;
}

// The evaluation pass on fixed configurations with the outputs of o (row
// i * n_meas + row for configuration i); reports device-side errors
// synchronously.  `validate` checks the configurations on the host first.
vp_status eval_configs(vp_ctx* ctx, Lattice* L, const int8_t* spins_dev, int32_t n_cfg, SampleOut o,
                       int32_t n_meas = 1, int32_t row = 0, bool validate = true) {
  if (!L->tensors_ready) return fail(ctx, VP_ERR_ARG, "tensors must be set first");
  if (n_cfg < 1 || n_cfg > L->p.n_chains) return fail(ctx, VP_ERR_ARG, "need 1 <= n_cfg <= n_chains");
  if (validate) {
    vp_status st = check_configs(ctx, *L, spins_dev, n_cfg);
    if (st != VP_OK) return st;
  }
  hipStream_t s = ctx->stream;
  // Evaluation reuses the chain slots; the sampler's state is invalidated.
  launch_copy_spins(L->dev, spins_dev, n_cfg, s);
  LatDev D = L->dev;
  D.n_chains = n_cfg;
  const vp_lattice& p = L->p;
  o.n_meas = n_meas;
  o.m = row;
  o.np_half = L->Np / 2;
  o.n_pairs = n_pairs_of(p);
  const bool cols = L->role == TWIN_COLUMNS;
  if (works_f64(p.prec)) run_eval<double>(D, o, n_cfg, s, !cols); else run_eval<float>(D, o, n_cfg, s, !cols);
  HIP_TRY(ctx, hipGetLastError());
  L->chains_ready = false;
  L->lower_valid = false;
  std::vector<ChainMeta> m(n_cfg), mc;
  if (cols) {
    // VP_VERT_COLUMN: the vertical terms from the transposed lattice's horizontal ones
    Lattice& C = ctx->lats[L->col];
    // the transposed configurations through the scratch (the copy clears their flags)
    launch_transpose_spins(L->spins, (int8_t*)C.d_sis, n_cfg, p.Ly, p.Lx, true, s);
    launch_copy_spins(C.dev, (const int8_t*)C.d_sis, n_cfg, s);
    LatDev Dt = C.dev;
    Dt.n_chains = n_cfg;
    SampleOut oc = scratch_out(C);
    const int npt = C.p.Ly * (C.p.Lx - 1) + (C.p.Ly - 1) * C.p.Lx;
    oc.n_pairs = npt;
    if (o.ratios) {
      if (!grow(s, C.col_ratios, sizeof(double) * (size_t)n_cfg * npt))
        return fail(ctx, VP_ERR_OOM, "column-wise ratio workspace");
      oc.ratios = (double*)C.col_ratios.p;
    }
    if (works_f64(p.prec)) run_eval<double>(Dt, oc, n_cfg, s, false); else run_eval<float>(Dt, oc, n_cfg, s, false);
    launch_add_energy(o.e_loc, n_meas, row, oc.e_loc, n_cfg, s);
    if (o.ratios) launch_column_ratios(oc.ratios, npt, o.ratios, o.n_pairs, n_cfg, p.Ly, p.Lx, s);
    HIP_TRY(ctx, hipGetLastError());
    mc.resize(n_cfg);
    HIP_TRY(ctx, hipMemcpyAsync(mc.data(), C.meta, sizeof(ChainMeta) * n_cfg, hipMemcpyDeviceToHost, s));
  } else if (L->role == TWIN_KNIGHTS) {
    const bool ok = works_f64(p.prec) ? eval_knights<double>(ctx, *L, n_cfg, o.e_loc, n_meas, row, o.ratios, o.n_pairs, s)
                                      : eval_knights<float>(ctx, *L, n_cfg, o.e_loc, n_meas, row, o.ratios, o.n_pairs, s);
    if (!ok) return fail(ctx, VP_ERR_OOM, "knight-bond ratio workspace");
    HIP_TRY(ctx, hipGetLastError());
    mc.resize(n_cfg);
    HIP_TRY(ctx, hipMemcpyAsync(mc.data(), ctx->lats[L->col].meta, sizeof(ChainMeta) * n_cfg, hipMemcpyDeviceToHost,
                                s));
  }
  HIP_TRY(ctx, hipMemcpyAsync(m.data(), L->meta, sizeof(ChainMeta) * n_cfg, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  for (size_t i = 0; i < mc.size(); ++i) m[i].flags |= mc[i].flags;
  for (int i = 0; i < n_cfg; ++i) {
    if (m[i].flags & FLAG_NONFINITE) return fail(ctx, VP_ERR_NONFINITE, "configuration %d: non-finite value", i);
    if (m[i].flags & FLAG_ZERO) return fail(ctx, VP_ERR_ZERO_AMPLITUDE, "configuration %d: zero amplitude", i);
  }
  return VP_OK;
}

// Workspace of one batched network call of n configurations, in the lattice's
// grow-only buffers.
struct NetWork {
  float* work = nullptr;
  double* part = nullptr;
  int* cnt = nullptr;
  double* scal = nullptr;
  float* grad = nullptr;
  int8_t* sb = nullptr;
  double* rb = nullptr;
  int32_t* idx = nullptr;
  bool alloc(Lattice& L, int n, hipStream_t s) {
    const int H = L.p.Ly, W = L.p.Lx;
    if (!(grow(s, L.nw_work, sizeof(float) * net_work_floats(n, H, W)) && grow(s, L.nw_part, sizeof(double) * n) &&
          grow(s, L.nw_cnt, sizeof(int) * n) && grow(s, L.nw_scal, sizeof(double) * 4) &&
          grow(s, L.nw_grad, sizeof(float) * NET_NPARAM) && grow(s, L.nw_sb, (size_t)n * H * W) &&
          grow(s, L.nw_rb, sizeof(double) * n * (H - 1) * (W - 1)) && grow(s, L.nw_idx, sizeof(int32_t) * n)))
      return false;
    work = (float*)L.nw_work.p; part = (double*)L.nw_part.p; cnt = (int*)L.nw_cnt.p;
    scal = (double*)L.nw_scal.p; grad = (float*)L.nw_grad.p; sb = (int8_t*)L.nw_sb.p;
    rb = (double*)L.nw_rb.p; idx = (int32_t*)L.nw_idx.p;
    return true;
  }
};

}  // namespace

extern "C" {

int64_t vp_num_params(const vp_lattice* p) {
  if (!p || p->Ly < 1 || p->Lx < 1 || p->D < 1) return -1;
  int64_t n = 0;
  for (int y = 0; y < p->Ly; ++y)
    for (int x = 0; x < p->Lx; ++x) {
      int32_t d[4];
      site_dims(*p, y, x, d);
      n += 2LL * d[0] * d[1] * d[2] * d[3];
    }
  return n;
}

int64_t vp_workspace_bytes(const vp_lattice* p) {
  if (!p) return -1;
  Plan P = plan_workspace(*p, nullptr);
  int64_t b = (int64_t)p->n_chains * (P.ws * (int64_t)type_size(p->prec) + P.cws * 8 + P.iws * 4 + P.dws * 8 +
                                      p->Ly * p->Lx + (int64_t)sizeof(ChainMeta));
  if (p->vertical == VP_VERT_COLUMN || has_knights(*p)) {  // the transposed lattice's chains
    const vp_lattice t = transposed_params(*p);
    Plan Q = plan_workspace(t, nullptr);
    b += (int64_t)t.n_chains * (Q.ws * (int64_t)type_size(t.prec) + Q.cws * 8 + Q.iws * 4 + Q.dws * 8 +
                                t.Ly * t.Lx + (int64_t)sizeof(ChainMeta));
  }
  return b;
}

const char* vp_last_error(const vp_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

vp_status vp_create(const vp_lattice* lats, int32_t n_lats, uint64_t seed, void* stream, vp_ctx** out) {
  if (!lats || n_lats < 1 || !out) return fail(nullptr, VP_ERR_ARG, "null argument or n_lats < 1");
  *out = nullptr;
  for (int i = 0; i < n_lats; ++i) {
    vp_status st = check_lattice(nullptr, lats[i]);
    if (st != VP_OK) return st;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(nullptr, VP_ERR_DEVICE, "no HIP device available");
  {
    // the allocation-free forward pass's scratch on this GPU: looked up once per device
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = net_scratch_setup(dev);
    if (e != hipSuccess)
      return fail(nullptr, VP_ERR_DEVICE, "static scratch lookup failed: %s", hipGetErrorString(e));
  }
  vp_ctx* ctx = new vp_ctx;
  ctx->seed = seed;
  ctx->stream = (hipStream_t)stream;
  // the caller's lattices, then the transposed lattice of each VP_VERT_COLUMN
  // one (Philox key word 1: its lattice index + 65536)
  std::vector<vp_lattice> all(lats, lats + n_lats);
  std::vector<int> key(n_lats), twin_role(n_lats, TWIN_NONE);
  for (int i = 0; i < n_lats; ++i) key[i] = i;
  ctx->n_user = n_lats;
  std::vector<std::pair<int, int>> twins;  // (lattice, role)
  for (int i = 0; i < n_lats; ++i) {
    const int role = lats[i].vertical == VP_VERT_COLUMN ? TWIN_COLUMNS : (has_knights(lats[i]) ? TWIN_KNIGHTS : 0);
    if (role == TWIN_NONE) continue;
    twins.push_back({i, role});
    all.push_back(transposed_params(lats[i]));
    key.push_back(i + 65536);
    twin_role.push_back(role);
  }
  ctx->lats.resize(all.size());
  for (size_t t = 0; t < twins.size(); ++t) {
    ctx->lats[twins[t].first].col = n_lats + (int)t;
    ctx->lats[twins[t].first].role = twins[t].second;
  }
  for (int i = 0; i < (int)all.size(); ++i) {
    Lattice& L = ctx->lats[i];
    L.p = all[i];
    const vp_lattice& p = L.p;
    L.N = p.Ly * p.Lx;
    L.tsize = type_size(p.prec);
    L.offs.assign(L.N + 1, 0);
    L.coff.assign(L.N + 1, 0);
    L.dims.assign(4 * L.N, 1);
    L.sizes.assign(L.N, 0);
    for (int k = 0; k < L.N; ++k) {
      site_dims(p, k / p.Lx, k % p.Lx, &L.dims[4 * k]);
      L.sizes[k] = L.dims[4 * k] * L.dims[4 * k + 1] * L.dims[4 * k + 2] * L.dims[4 * k + 3];
      L.offs[k + 1] = L.offs[k] + 2LL * L.sizes[k];
      L.coff[k + 1] = L.coff[k] + L.sizes[k];
    }
    L.Np = L.offs[L.N];
    plan_bonds(L);
    Plan P = plan_workspace(p, &L.dev);
    const int64_t d4 = (int64_t)p.D * p.D * p.D * p.D;
    auto alloc = [&](void** ptr, size_t bytes) -> bool { return hipMalloc(ptr, std::max<size_t>(bytes, 64)) == hipSuccess; };
    bool ok = alloc((void**)&L.T, sizeof(double) * L.Np) && alloc(&L.Tw, L.tsize * L.N * 2 * d4) &&
              alloc(&L.ws, L.tsize * P.ws * p.n_chains) && alloc((void**)&L.cws, 8 * P.cws * p.n_chains) &&
              alloc((void**)&L.iws, 4 * P.iws * p.n_chains) &&
              alloc((void**)&L.dws, 8 * P.dws * p.n_chains) &&
              alloc((void**)&L.meta, sizeof(ChainMeta) * p.n_chains) &&
              alloc((void**)&L.spins, (size_t)p.n_chains * L.N) &&
              alloc((void**)&L.d_kU, 4 * L.kU.size()) && alloc((void**)&L.d_kD, 4 * L.kD.size()) &&
              alloc((void**)&L.d_dims, 4 * L.dims.size()) && alloc((void**)&L.d_sizes, 4 * L.sizes.size()) &&
              alloc((void**)&L.d_offs, 8 * L.offs.size()) && alloc((void**)&L.d_coff, 8 * L.coff.size()) &&
              alloc((void**)&L.d_scratch, 64 * sizeof(double)) &&
              alloc((void**)&L.d_net, sizeof(float) * NET_NPARAM) &&
              alloc((void**)&L.d_net64, sizeof(double) * NET_NPARAM) &&
              alloc((void**)&L.d_netbf, NET_BF_BYTES) &&
              alloc((void**)&L.d_adam, 2 * sizeof(float) * NET_NPARAM) &&
              alloc((void**)&L.d_sis, sis_bytes(p));
    if (!ok) {
      vp_destroy(ctx);
      return fail(nullptr, VP_ERR_OOM, "device allocation failed for lattice %d", i);
    }
    hipMemcpy(L.d_kU, L.kU.data(), 4 * L.kU.size(), hipMemcpyHostToDevice);
    hipMemcpy(L.d_kD, L.kD.data(), 4 * L.kD.size(), hipMemcpyHostToDevice);
    hipMemcpy(L.d_dims, L.dims.data(), 4 * L.dims.size(), hipMemcpyHostToDevice);
    hipMemcpy(L.d_sizes, L.sizes.data(), 4 * L.sizes.size(), hipMemcpyHostToDevice);
    hipMemcpy(L.d_offs, L.offs.data(), 8 * L.offs.size(), hipMemcpyHostToDevice);
    hipMemcpy(L.d_coff, L.coff.data(), 8 * L.coff.size(), hipMemcpyHostToDevice);
    hipMemset(L.ws, 0, L.tsize * P.ws * p.n_chains);
    hipMemset(L.cws, 0, 8 * P.cws * p.n_chains);
    hipMemset(L.iws, 0, 4 * P.iws * p.n_chains);
    hipMemset(L.dws, 0, 8 * P.dws * p.n_chains);
    hipMemset(L.meta, 0, sizeof(ChainMeta) * p.n_chains);
    hipMemset(L.spins, 0, (size_t)p.n_chains * L.N);
    LatDev& D = L.dev;
    D.Ly = p.Ly; D.Lx = p.Lx; D.d = p.D; D.c = p.Dc; D.N = L.N;
    D.J1 = p.J1; D.Jd = diag_coupling(p); D.Ja = anti_coupling(p); D.n_chains = p.n_chains;
    D.Jk = has_knights(p) ? p.J2 : 0.0;
    if (twin_role[i] == TWIN_KNIGHTS) {  // evaluates the knight bonds (y,x)-(y+1,x+2) alone
      D.J1 = 0.0; D.Jd = 0.0; D.Ja = 0.0;
    }
    D.seed = seed; D.lat_id = key[i];
    D.cmode = p.compress; D.fit_sweeps = p.fit_sweeps;
    D.Tw = L.Tw; D.ws = L.ws; D.ws_stride = P.ws;
    D.cws = L.cws; D.cws_stride = P.cws;
    D.iws = L.iws; D.iws_stride = P.iws; D.dws = L.dws; D.dws_stride = P.dws;
    D.meta = L.meta; D.spins = L.spins;
    D.trace = nullptr;
    D.net = works_f64(p.prec) ? (const void*)L.d_net64 : (const void*)L.d_net;
    D.net_bf = (const void*)L.d_netbf;
    D.n_bonds = p.Ly * (p.Lx - 1) + (p.Ly - 1) * p.Lx;
    D.kU = L.d_kU; D.kD = L.d_kD; D.dims = L.d_dims; D.coff = L.d_coff;
    if (works_f64(p.prec)) launch_init_trivial<double>(D, ctx->stream);
    else launch_init_trivial<float>(D, ctx->stream);
    if (hipGetLastError() != hipSuccess) {
      vp_destroy(ctx);
      return fail(nullptr, VP_ERR_DEVICE, "kernel launch failed while creating the context");
    }
  }
  *out = ctx;
  return VP_OK;
}

vp_status vp_destroy(vp_ctx* ctx) {
  if (!ctx) return VP_OK;
  if (ctx->stream) hipStreamSynchronize(ctx->stream); else hipDeviceSynchronize();
  for (hipEvent_t e : ctx->ev) hipEventDestroy(e);
  for (auto& L : ctx->lats) {
    void* ptrs[] = {L.T, L.Tw, L.ws, L.cws, L.iws, L.dws, L.meta, L.spins, L.d_kU, L.d_kD,
                    L.d_dims, L.d_sizes, L.d_offs, L.d_coff, L.d_scratch, L.d_net, L.d_net64, L.d_adam,
                    L.d_sis, L.d_netbf};
    for (void* q : ptrs)
      if (q) hipFree(q);
    Lattice::Buf* bufs[] = {&L.sr_work, &L.sr_flag, &L.opt_lp, &L.opt_el, &L.opt_grad, &L.opt_em, &L.opt_sg,
                            &L.opt_so, &L.opt_dl, &L.nw_work, &L.nw_part, &L.nw_cnt, &L.nw_scal, &L.nw_grad,
                            &L.nw_sb, &L.nw_rb, &L.nw_idx, &L.su_B, &L.su_lam, &L.su_change, &L.su_scr,
                            &L.col_ratios};
    for (Lattice::Buf* b : bufs)
      if (b->p) hipFree(b->p);
  }
  void* qp[] = {ctx->q_lats, ctx->q_outs, ctx->q_items, ctx->q_next};
  for (void* q : qp)
    if (q) hipFree(q);
  if (ctx->cap_event) hipEventDestroy(ctx->cap_event);
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  delete ctx;
  return VP_OK;
}

static vp_status stage_tensors(vp_ctx* ctx, Lattice& L) {
  if (works_f64(L.p.prec))
    launch_prepare_tensors<double>(L.dev, L.T, (double*)L.Tw, L.d_offs, ctx->stream);
  else
    launch_prepare_tensors<float>(L.dev, L.T, (float*)L.Tw, L.d_offs, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  L.tensors_ready = true;
  L.lower_valid = false;
  L.su_valid = false;
  if (L.col >= 0) {  // the transposed lattice carries the same state
    Lattice& C = ctx->lats[L.col];
    launch_transpose_tensors(L.T, C.T, L.d_offs, C.d_offs, L.d_dims, L.p.Ly, L.p.Lx, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
    return stage_tensors(ctx, C);
  }
  return VP_OK;
}

vp_status vp_set_tensors(vp_ctx* ctx, int32_t lat, const double* T_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !T_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null tensor pointer");
  HIP_TRY(ctx, hipMemcpyAsync(L->T, T_dev, sizeof(double) * L->Np, hipMemcpyDeviceToDevice, ctx->stream));
  return stage_tensors(ctx, *L);
}

vp_status vp_simple_update(vp_ctx* ctx, int32_t lat, double dt, int32_t n_steps, double* change_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (!std::isfinite(dt) || n_steps < 0) return fail(ctx, VP_ERR_ARG, "dt must be finite and n_steps >= 0");
  if (!L->tensors_ready) return fail(ctx, VP_ERR_ARG, "tensors must be set first");
  hipStream_t s = ctx->stream;
  const int Ly = L->p.Ly, Lx = L->p.Lx, D = L->p.D;
  const bool nnn = has_diagonals(L->p);
  const double Jdiag[2] = {diag_coupling(L->p), anti_coupling(L->p)};
  const int nl = Ly * (Lx - 1) + (Ly - 1) * Lx;
  int most = 1;
  for (int c = 0; c < 4; ++c) {
    most = std::max(most, su_class_links(Ly, Lx, c));
    if (nnn) most = std::max(most, su_class_plaquettes(Ly, Lx, c));
  }
  const int64_t stride = su_scratch_doubles(D, nnn);
  // work-groups per launch: every link or plaquette of a class, within about 1 GiB of scratch
  const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)most, 512, ((int64_t)1 << 27) / stride}));
  if (!(grow(s, L->su_B, sizeof(double) * L->Np) && grow(s, L->su_lam, sizeof(double) * std::max(nl, 1) * D) &&
        grow(s, L->su_change, sizeof(double) * std::max(nl, 1) * D) &&
        grow(s, L->su_scr, sizeof(double) * (size_t)chunk * stride)))
    return fail(ctx, VP_ERR_OOM, "simple-update workspace");
  double* B = (double*)L->su_B.p;
  double* lam = (double*)L->su_lam.p;
  double* prev = (double*)L->su_change.p;  // the lambdas at the start of a step
  double* scr = (double*)L->su_scr.p;
  if (!L->su_valid) {  // start: the current tensors, every lambda 1
    HIP_TRY(ctx, hipMemcpyAsync(B, L->T, sizeof(double) * L->Np, hipMemcpyDeviceToDevice, s));
    if (nl > 0) launch_su_init(lam, (int64_t)nl * D, s);
  }
  for (int step = 0; step < n_steps; ++step) {
    if (change_dev && nl > 0)
      HIP_TRY(ctx, hipMemcpyAsync(prev, lam, sizeof(double) * nl * D, hipMemcpyDeviceToDevice, s));
    for (int c = 0; c < 4; ++c) {
      const int count = su_class_links(Ly, Lx, c);
      for (int first = 0; first < count; first += chunk)
        launch_su_class(B, lam, L->d_offs, L->d_dims, Ly, Lx, D, c, first, std::min(chunk, count - first), dt,
                        L->p.J1, scr, stride, s);
    }
    if (nnn)
      for (int c = 0; c < 4; ++c)
        for (int anti = 0; anti < 2; ++anti) {
          if (Jdiag[anti] == 0.0) continue;  // an uncoupled diagonal (triangular lattice)
          const int count = su_class_plaquettes(Ly, Lx, c);
          for (int first = 0; first < count; first += chunk)
            launch_su_nnn(B, lam, L->d_offs, L->d_dims, Ly, Lx, D, c, anti, first, std::min(chunk, count - first),
                          dt, Jdiag[anti], scr, stride, s);
        }
    if (change_dev) launch_su_mean(lam, prev, nl, D, change_dev + step, s);
    HIP_TRY(ctx, hipGetLastError());
  }
  launch_su_absorb(B, lam, L->d_offs, L->d_dims, Ly, Lx, D, L->T, s);
  HIP_TRY(ctx, hipGetLastError());
  vp_status st = stage_tensors(ctx, *L);
  if (st != VP_OK) return st;
  L->su_valid = true;  // a later call continues from B and the lambdas
  return VP_OK;
}

vp_status vp_simple_update_lambdas(vp_ctx* ctx, int32_t lat, double* lam_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !lam_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (!L->su_valid) return fail(ctx, VP_ERR_ARG, "no simple update of the current tensors");
  const int nl = L->p.Ly * (L->p.Lx - 1) + (L->p.Ly - 1) * L->p.Lx;
  if (nl > 0)
    HIP_TRY(ctx, hipMemcpyAsync(lam_dev, L->su_lam.p, sizeof(double) * nl * L->p.D, hipMemcpyDeviceToDevice,
                                ctx->stream));
  return VP_OK;
}

vp_status vp_get_tensors(vp_ctx* ctx, int32_t lat, double* T_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !T_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null tensor pointer");
  HIP_TRY(ctx, hipMemcpyAsync(T_dev, L->T, sizeof(double) * L->Np, hipMemcpyDeviceToDevice, ctx->stream));
  return VP_OK;
}

vp_status vp_init_tensors(vp_ctx* ctx, int32_t lat, uint64_t seed, double scale, double perturb) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (!(scale > 0)) scale = 1.0 / ((double)L->p.D * L->p.D);
  launch_init_tensors(L->T, L->Np, seed, lat, scale, perturb, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  return stage_tensors(ctx, *L);
}

vp_status vp_init_chains(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (spins_dev) {
    std::vector<int8_t> h((size_t)L->p.n_chains * L->N);
    HIP_TRY(ctx, hipMemcpyAsync(h.data(), spins_dev, h.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int ch = 0; ch < L->p.n_chains; ++ch) {
      int up = 0;
      for (int i = 0; i < L->N; ++i) {
        int8_t v = h[(size_t)ch * L->N + i];
        if (v != 0 && v != 1) return fail(ctx, VP_ERR_SHAPE, "spins must be 0 or 1");
        up += v;
      }
      if (2 * up != L->N) return fail(ctx, VP_ERR_SHAPE, "chain %d is not in the S^z_tot = 0 sector", ch);
    }
    HIP_TRY(ctx, hipMemcpyAsync(L->spins, spins_dev, h.size(), hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(L->meta, 0, sizeof(ChainMeta) * L->p.n_chains, ctx->stream));
  } else {
    launch_init_chains(L->dev, ctx->stream);
    HIP_TRY(ctx, hipGetLastError());
  }
  L->chains_ready = true;
  L->sweeps = 0;
  L->lower_valid = false;
  if (L->col >= 0)  // the transposed lattice's sweep and move counters follow the chains
    HIP_TRY(ctx, hipMemsetAsync(ctx->lats[L->col].meta, 0, sizeof(ChainMeta) * L->p.n_chains, ctx->stream));
  return VP_OK;
}

vp_status vp_sample(vp_ctx* ctx, int32_t lat, int32_t n_burn, int32_t n_meas, double* log_abs_psi_dev,
                    int8_t* sign_dev, double* e_loc_dev, void* dlnpsi_dev, int8_t* spins_out_dev,
                    int64_t* accept_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (n_burn < 0 || n_meas < 0) return fail(ctx, VP_ERR_ARG, "negative sweep count");
  if (!L->tensors_ready || !L->chains_ready)
    return fail(ctx, VP_ERR_ARG, "tensors and chains must be initialised first");
  if (n_meas > 0 && (!log_abs_psi_dev || !sign_dev || !e_loc_dev))
    return fail(ctx, VP_ERR_ARG, "log_abs_psi, sign and e_loc outputs are required");
  hipStream_t s = ctx->stream;
  const bool f64 = works_f64(L->p.prec);
  if (L->sampler == VP_SAMPLER_SIS_PAIR) {
    if (L->schedule != VP_SCHED_PHASES)
      return fail(ctx, VP_ERR_UNSUPPORTED, "the |Phi|^2 sampler runs the per-phase schedule only");
    if (dlnpsi_dev) return fail(ctx, VP_ERR_UNSUPPORTED, "the |Phi|^2 sampler produces no log-derivatives");
    vp_status st = f64 ? run_pair_sample<double>(ctx, *L, n_burn, n_meas, log_abs_psi_dev, sign_dev, e_loc_dev,
                                                  spins_out_dev)
                       : run_pair_sample<float>(ctx, *L, n_burn, n_meas, log_abs_psi_dev, sign_dev, e_loc_dev,
                                                spins_out_dev);
    if (st != VP_OK) return st;
    L->sweeps += n_burn + n_meas;
    if (accept_dev)
      HIP_TRY(ctx, hipMemcpy2DAsync(accept_dev, 2 * sizeof(int64_t), (const char*)L->meta + sizeof(int64_t),
                                    sizeof(ChainMeta), 2 * sizeof(int64_t), L->p.n_chains / 2,
                                    hipMemcpyDeviceToDevice, s));
    return VP_OK;
  }
  if (L->role == TWIN_KNIGHTS && L->schedule != VP_SCHED_PHASES)
    return fail(ctx, VP_ERR_UNSUPPORTED, "the triangular knight bonds are measured with the per-phase schedule only");
  if (L->role == TWIN_COLUMNS) {
    if (L->schedule != VP_SCHED_PHASES)
      return fail(ctx, VP_ERR_UNSUPPORTED, "column-wise vertical bonds run the per-phase schedule only");
    Lattice& C = ctx->lats[L->col];
    SampleOut o{};
    o.log_abs_psi = log_abs_psi_dev;
    o.sign = sign_dev;
    o.e_loc = e_loc_dev;
    o.dlnpsi = dlnpsi_dev;
    o.spins = spins_out_dev;
    o.n_meas = n_meas;
    o.m = 0;
    o.dyn_m = 1;  // row = sweep counter - (counter at the first measured sweep)
    o.sweep0 = L->sweeps + n_burn;
    o.np_half = L->Np / 2;
    vp_status st = f64 ? run_col_sample<double>(ctx, *L, C, n_burn, n_meas, o)
                       : run_col_sample<float>(ctx, *L, C, n_burn, n_meas, o);
    if (st != VP_OK) return st;
    L->sweeps += n_burn + n_meas;
    if (accept_dev) {  // the row pass's counts plus the column pass's
      HIP_TRY(ctx, hipMemcpy2DAsync(accept_dev, 2 * sizeof(int64_t), (const char*)L->meta + sizeof(int64_t),
                                    sizeof(ChainMeta), 2 * sizeof(int64_t), L->p.n_chains, hipMemcpyDeviceToDevice,
                                    s));
      launch_add_counts(C.meta, accept_dev, 2, L->p.n_chains, s);
    }
    HIP_TRY(ctx, hipGetLastError());
    return VP_OK;
  }
  if (!L->lower_valid) {
    if (f64) run_lower_pass<double>(ctx, *L, s); else run_lower_pass<float>(ctx, *L, s);
    L->lower_valid = true;
  }
  SampleOut o{};
  o.log_abs_psi = log_abs_psi_dev;
  o.sign = sign_dev;
  o.e_loc = e_loc_dev;
  o.dlnpsi = dlnpsi_dev;
  o.spins = spins_out_dev;
  o.ratios = nullptr;
  o.n_meas = n_meas;
  o.np_half = L->Np / 2;
  o.psi_meas = L->p.prec == VP_BF16;
  // measurement row = sweep counter - (counter at the first measured sweep)
  o.dyn_m = 1;
  o.sweep0 = L->sweeps + n_burn;
  vp_status st = VP_OK;
  if (L->schedule == VP_SCHED_PERSISTENT) {
    std::vector<Lattice*> one{L};
    std::vector<SampleOut> oo{o};
    st = f64 ? run_queue<double>(ctx, one, n_burn, n_meas, oo, s) : run_queue<float>(ctx, one, n_burn, n_meas, oo, s);
  } else if (L->schedule == VP_SCHED_GRAPH) {
    st = f64 ? run_graph<double>(ctx, *L, n_burn, n_meas, o, s) : run_graph<float>(ctx, *L, n_burn, n_meas, o, s);
  } else {
    for (int i = 0; i < n_burn + n_meas; ++i) {
      const SampleOut* op = i >= n_burn ? &o : nullptr;
      if (f64) run_sweep<double>(ctx, *L, op, s); else run_sweep<float>(ctx, *L, op, s);
      if (op && L->role == TWIN_KNIGHTS) {  // the knight bonds (y,x)-(y+2,x+1) of the final configurations
        const bool ok = f64 ? eval_knights<double>(ctx, *L, L->p.n_chains, e_loc_dev, n_meas, i - n_burn, nullptr, 0, s)
                            : eval_knights<float>(ctx, *L, L->p.n_chains, e_loc_dev, n_meas, i - n_burn, nullptr, 0, s);
        if (!ok) return fail(ctx, VP_ERR_OOM, "knight-bond workspace");
      }
      HIP_TRY(ctx, hipGetLastError());
    }
  }
  if (st != VP_OK) return st;
  L->sweeps += n_burn + n_meas;
  if (accept_dev) {
    // accepted / proposed pairs are the 2nd and 3rd int64 of ChainMeta
    HIP_TRY(ctx, hipMemcpy2DAsync(accept_dev, 2 * sizeof(int64_t), (const char*)L->meta + sizeof(int64_t),
                                  sizeof(ChainMeta), 2 * sizeof(int64_t), L->p.n_chains, hipMemcpyDeviceToDevice, s));
  }
  return VP_OK;
}

vp_status vp_set_schedule(vp_ctx* ctx, int32_t lat, int32_t schedule) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (schedule != VP_SCHED_PHASES && schedule != VP_SCHED_PERSISTENT && schedule != VP_SCHED_GRAPH)
    return fail(ctx, VP_ERR_ARG, "unknown schedule %d", schedule);
  L->schedule = schedule;
  return VP_OK;
}

vp_status vp_set_tile(vp_ctx* ctx, int32_t lat, int32_t tile) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (tile < 0 || tile >= VP_N_TILES) return fail(ctx, VP_ERR_ARG, "unknown tile variant %d", tile);
  L->dev.tile = tile;
  return VP_OK;
}

vp_status vp_sample_batch(vp_ctx* ctx, int32_t n_lats, const int32_t* lats_host, int32_t n_burn, int32_t n_meas,
                          const vp_outputs* outs_host) {
  if (!ctx || n_lats < 1 || !lats_host) return fail(ctx, VP_ERR_ARG, "need at least one lattice");
  if (n_burn < 0 || n_meas < 0) return fail(ctx, VP_ERR_ARG, "negative sweep count");
  if (n_meas > 0 && !outs_host) return fail(ctx, VP_ERR_ARG, "outputs are required for measured sweeps");
  std::vector<Lattice*> ls;
  std::vector<SampleOut> os;
  for (int i = 0; i < n_lats; ++i) {
    Lattice* L = get_lat(ctx, lats_host[i]);
    if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index %d", lats_host[i]);
    for (Lattice* q : ls)
      if (q == L) return fail(ctx, VP_ERR_ARG, "lattice %d listed twice", lats_host[i]);
    if (!L->tensors_ready || !L->chains_ready)
      return fail(ctx, VP_ERR_ARG, "lattice %d: tensors and chains must be initialised first", lats_host[i]);
    if (L->sampler == VP_SAMPLER_SIS_PAIR)
      return fail(ctx, VP_ERR_UNSUPPORTED, "lattice %d: the |Phi|^2 sampler runs through vp_sample only", lats_host[i]);
    if (L->col >= 0)
      return fail(ctx, VP_ERR_UNSUPPORTED,
                  "lattice %d: column-wise vertical bonds and the triangular knight bonds run through vp_sample only",
                  lats_host[i]);
    if (!ls.empty() && (L->p.D != ls[0]->p.D || L->p.Dc != ls[0]->p.Dc || L->p.prec != ls[0]->p.prec))
      return fail(ctx, VP_ERR_SHAPE, "one batch needs equal D, Dc and precision");
    SampleOut o{};
    if (n_meas > 0) {
      const vp_outputs& u = outs_host[i];
      if (!u.log_abs_psi_dev || !u.sign_dev || !u.e_loc_dev)
        return fail(ctx, VP_ERR_ARG, "lattice %d: log_abs_psi, sign and e_loc outputs are required", lats_host[i]);
      o.log_abs_psi = u.log_abs_psi_dev;
      o.sign = u.sign_dev;
      o.e_loc = u.e_loc_dev;
      o.dlnpsi = u.dlnpsi_dev;
      o.spins = u.spins_out_dev;
    }
    o.n_meas = n_meas;
    o.np_half = L->Np / 2;
    o.psi_meas = L->p.prec == VP_BF16;
    o.dyn_m = 1;
    o.sweep0 = L->sweeps + n_burn;
    ls.push_back(L);
    os.push_back(o);
  }
  hipStream_t s = ctx->stream;
  const bool f64 = works_f64(ls[0]->p.prec);
  for (Lattice* L : ls)
    if (!L->lower_valid) {
      if (f64) run_lower_pass<double>(ctx, *L, s); else run_lower_pass<float>(ctx, *L, s);
      L->lower_valid = true;
    }
  vp_status st = f64 ? run_queue<double>(ctx, ls, n_burn, n_meas, os, s) : run_queue<float>(ctx, ls, n_burn, n_meas, os, s);
  if (st != VP_OK) return st;
  for (Lattice* L : ls) L->sweeps += n_burn + n_meas;
  return VP_OK;
}

vp_status vp_autotune(vp_ctx* ctx, int32_t lat, int32_t sweeps, double* ms_host, int32_t* schedule_out) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (sweeps < 1) return fail(ctx, VP_ERR_ARG, "sweeps must be >= 1");
  if (!L->tensors_ready || !L->chains_ready)
    return fail(ctx, VP_ERR_ARG, "tensors and chains must be initialised first");
  hipStream_t s = ctx->stream;
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  const int32_t cand[3] = {VP_SCHED_PHASES, VP_SCHED_PERSISTENT, VP_SCHED_GRAPH};
  double best = 1e300;
  int32_t pick = VP_SCHED_PHASES;
  const bool timing = ctx->timing;
  ctx->timing = false;
  vp_status st = VP_OK;
  for (int k = 0; k < 3 && st == VP_OK; ++k) {
    if (cand[k] == VP_SCHED_PERSISTENT && L->p.compress != VP_COMPRESS_CANONICAL) {
      if (ms_host) ms_host[k] = -1.0;  // not available with the variational fit
      continue;
    }
    if (cand[k] != VP_SCHED_PHASES && (L->col >= 0 || L->sampler == VP_SAMPLER_SIS_PAIR)) {
      if (ms_host) ms_host[k] = -1.0;  // the per-phase schedule only
      continue;
    }
    L->schedule = cand[k];
    // one untimed sweep first (initial boundaries, graph and code warm-up)
    st = vp_sample(ctx, lat, 1, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (st != VP_OK) break;
    hipEventRecord(e0, s);
    st = vp_sample(ctx, lat, sweeps, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    hipEventRecord(e1, s);
    if (st != VP_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) { st = fail(ctx, VP_ERR_DEVICE, "autotune timing failed"); break; }
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms_host) ms_host[k] = ms / sweeps;
    if (ms < best) { best = ms; pick = cand[k]; }
  }
  ctx->timing = timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != VP_OK) return st;
  L->schedule = pick;
  if (schedule_out) *schedule_out = pick;
  return VP_OK;
}

vp_status vp_autotune_tiles(vp_ctx* ctx, int32_t lat, int32_t sweeps, double* ms_host, int32_t* tile_out) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (sweeps < 1) return fail(ctx, VP_ERR_ARG, "sweeps must be >= 1");
  if (!L->tensors_ready || !L->chains_ready)
    return fail(ctx, VP_ERR_ARG, "tensors and chains must be initialised first");
  hipStream_t s = ctx->stream;
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  double best = 1e300;
  int32_t pick = VP_TILE_DEFAULT;
  const bool timing = ctx->timing;
  ctx->timing = false;
  vp_status st = VP_OK;
  for (int k = 0; k < VP_N_TILES && st == VP_OK; ++k) {
    L->dev.tile = k;
    st = vp_sample(ctx, lat, 1, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);  // warm-up
    if (st != VP_OK) break;
    hipEventRecord(e0, s);
    st = vp_sample(ctx, lat, sweeps, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    hipEventRecord(e1, s);
    if (st != VP_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) { st = fail(ctx, VP_ERR_DEVICE, "autotune timing failed"); break; }
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms_host) ms_host[k] = ms / sweeps;
    if (ms < best) { best = ms; pick = k; }
  }
  ctx->timing = timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  L->dev.tile = pick;
  if (st != VP_OK) return st;
  if (tile_out) *tile_out = pick;
  return VP_OK;
}

vp_status vp_trace_ratios(vp_ctx* ctx, int32_t lat, double* trace_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (L->role == TWIN_COLUMNS) return fail(ctx, VP_ERR_UNSUPPORTED, "no ratio trace with column-wise vertical bonds");
  L->dev.trace = trace_dev;
  return VP_OK;
}

vp_status vp_eval(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n_cfg, double* log_abs_psi_dev,
                  int8_t* sign_dev, double* e_loc_dev, void* dlnpsi_dev, double* ratios_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !spins_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null spins");
  if (!log_abs_psi_dev || !sign_dev || !e_loc_dev) return fail(ctx, VP_ERR_ARG, "null output pointer");
  SampleOut o{};
  o.log_abs_psi = log_abs_psi_dev;
  o.sign = sign_dev;
  o.e_loc = e_loc_dev;
  o.dlnpsi = dlnpsi_dev;
  o.ratios = ratios_dev;
  return eval_configs(ctx, L, spins_dev, n_cfg, o);
}

vp_status vp_eval_sis(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n_cfg, double* log_abs_phi_dev,
                      int8_t* sign_phi_dev, double* e_loc_phi_dev, double* log_w_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !spins_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null spins");
  if (!log_abs_phi_dev || !sign_phi_dev || !e_loc_phi_dev || !log_w_dev)
    return fail(ctx, VP_ERR_ARG, "null output pointer");
  if (n_cfg < 1 || n_cfg > L->p.n_chains) return fail(ctx, VP_ERR_ARG, "need 1 <= n_cfg <= n_chains");
  hipStream_t s = ctx->stream;
  const size_t nb = (size_t)n_cfg * L->N;
  // the scratch reserved at vp_create (sized for n_chains configurations):
  // reversed configurations, then log|Psi(Sbar)|, E_loc(Sbar), sign(Sbar)
  char* work = L->d_sis;
  const size_t off_l = (nb + 255) / 256 * 256, off_e = off_l + sizeof(double) * n_cfg,
               off_s = off_e + sizeof(double) * n_cfg;
  int8_t* rev = (int8_t*)work;
  double* lr = (double*)(work + off_l);
  double* er = (double*)(work + off_e);
  int8_t* sr = (int8_t*)(work + off_s);
  // S into the caller's outputs, Sbar into the workspace, then combined in place
  vp_status st = vp_eval(ctx, lat, spins_dev, n_cfg, log_abs_phi_dev, sign_phi_dev, e_loc_phi_dev, nullptr, nullptr);
  if (st == VP_OK) {
    launch_reverse_spins(spins_dev, rev, (int64_t)nb, s);
    st = vp_eval(ctx, lat, rev, n_cfg, lr, sr, er, nullptr, nullptr);
  }
  if (st == VP_OK) {
    launch_sis_combine(n_cfg, log_abs_phi_dev, sign_phi_dev, e_loc_phi_dev, lr, sr, er, log_w_dev, s);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      st = fail(ctx, VP_ERR_DEVICE, "symmetrisation kernel failed");
  }
  hipStreamSynchronize(s);
  return st;
}

vp_status vp_sample_split(vp_ctx* ctx, int32_t lat_sample, int32_t lat_measure, int32_t n_burn, int32_t n_meas,
                          double* log_abs_psi_dev, int8_t* sign_dev, double* e_loc_dev, void* dlnpsi_dev,
                          int8_t* spins_out_dev) {
  Lattice* A = get_lat(ctx, lat_sample);
  Lattice* M = get_lat(ctx, lat_measure);
  if (!A || !M || lat_sample == lat_measure) return fail(ctx, VP_ERR_ARG, "need two distinct lattice indices");
  if (n_burn < 0 || n_meas < 0) return fail(ctx, VP_ERR_ARG, "negative sweep count");
  const vp_lattice& pa = A->p;
  const vp_lattice& pm = M->p;
  if (pa.Ly != pm.Ly || pa.Lx != pm.Lx || pa.D != pm.D || pa.J1 != pm.J1 || pa.J2 != pm.J2 || pa.prec != pm.prec ||
      pa.geometry != pm.geometry)
    return fail(ctx, VP_ERR_SHAPE, "the sampling and measuring lattices may differ only in Dc and chain count");
  if (pm.n_chains < pa.n_chains)
    return fail(ctx, VP_ERR_SHAPE, "the measuring lattice needs at least as many chains as the sampling one");
  if (!A->tensors_ready || !A->chains_ready || !M->tensors_ready)
    return fail(ctx, VP_ERR_ARG, "tensors of both lattices and the sampling chains must be set first");
  if (A->sampler == VP_SAMPLER_SIS_PAIR)
    return fail(ctx, VP_ERR_UNSUPPORTED, "the |Phi|^2 sampler runs through vp_sample only");
  if (A->col >= 0 || M->col >= 0)
    return fail(ctx, VP_ERR_UNSUPPORTED,
                "column-wise vertical bonds and the triangular knight bonds run through vp_sample and vp_eval only");
  if (n_meas > 0 && (!log_abs_psi_dev || !sign_dev || !e_loc_dev))
    return fail(ctx, VP_ERR_ARG, "log_abs_psi, sign and e_loc outputs are required");
  hipStream_t s = ctx->stream;
  const bool f64 = works_f64(pa.prec);
  if (!A->lower_valid) {
    if (f64) run_lower_pass<double>(ctx, *A, s); else run_lower_pass<float>(ctx, *A, s);
    A->lower_valid = true;
  }
  for (int i = 0; i < n_burn + n_meas; ++i) {
    // a sweep at the sampling cutoff (its bottom-up pass rebuilds the lower
    // boundaries the next sweep needs), then the chains' states measured at
    // the measuring cutoff
    if (f64) run_sweep<double>(ctx, *A, nullptr, s); else run_sweep<float>(ctx, *A, nullptr, s);
    HIP_TRY(ctx, hipGetLastError());
    if (i >= n_burn) {
      SampleOut o{};
      o.log_abs_psi = log_abs_psi_dev;
      o.sign = sign_dev;
      o.e_loc = e_loc_dev;
      o.dlnpsi = dlnpsi_dev;
      o.spins = spins_out_dev;
      vp_status st = eval_configs(ctx, M, A->spins, pa.n_chains, o, n_meas, i - n_burn, false);
      if (st != VP_OK) return st;
    }
  }
  A->sweeps += n_burn + n_meas;
  return check_flags(ctx, *A);
}

vp_status vp_plaquette_ratios(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n_cfg,
                              double* ratios_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !spins_dev || !ratios_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (L->p.Ly < 2 || L->p.Lx < 2) return fail(ctx, VP_ERR_SHAPE, "plaquettes need Ly, Lx >= 2");
  SampleOut o{};
  o.plaq = ratios_dev;
  return eval_configs(ctx, L, spins_dev, n_cfg, o);
}

int64_t vp_proposal_num_params(void) { return NET_NPARAM; }

vp_status vp_proposal_set_weights(vp_ctx* ctx, int32_t lat, const float* w_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !w_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  hipStream_t s = ctx->stream;
  HIP_TRY(ctx, hipMemcpyAsync(L->d_net, w_dev, sizeof(float) * NET_NPARAM, hipMemcpyDeviceToDevice, s));
  net_cast_f64(L->d_net, L->d_net64, s);
  net_pack_bf16(L->d_net, L->d_netbf, s);
  HIP_TRY(ctx, hipMemsetAsync(L->d_adam, 0, 2 * sizeof(float) * NET_NPARAM, s));
  HIP_TRY(ctx, hipGetLastError());
  L->adam_t = 0;
  L->net_ready = true;
  return VP_OK;
}

vp_status vp_proposal_get_weights(vp_ctx* ctx, int32_t lat, float* w_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !w_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (!L->net_ready) return fail(ctx, VP_ERR_ARG, "the proposal network has no weights yet");
  HIP_TRY(ctx, hipMemcpyAsync(w_dev, L->d_net, sizeof(float) * NET_NPARAM, hipMemcpyDeviceToDevice, ctx->stream));
  return VP_OK;
}

vp_status vp_set_sampler(vp_ctx* ctx, int32_t lat, int32_t sampler) {
  Lattice* L = get_lat(ctx, lat);
  if (!L) return fail(ctx, VP_ERR_ARG, "bad lattice index");
  if (sampler != VP_SAMPLER_PAIR_SEQ && sampler != VP_SAMPLER_LEARNED_PLAQ && sampler != VP_SAMPLER_SIS_PAIR)
    return fail(ctx, VP_ERR_ARG, "unknown sampler %d", sampler);
  if (sampler == VP_SAMPLER_SIS_PAIR && L->p.n_chains % 2)
    return fail(ctx, VP_ERR_SHAPE, "the |Phi|^2 sampler pairs the chains: n_chains must be even");
  if (sampler != VP_SAMPLER_PAIR_SEQ && L->role == TWIN_COLUMNS)
    return fail(ctx, VP_ERR_UNSUPPORTED, "column-wise vertical bonds run the pair sampler only");
  if (sampler == VP_SAMPLER_SIS_PAIR && L->role == TWIN_KNIGHTS)
    return fail(ctx, VP_ERR_UNSUPPORTED, "the |Phi|^2 chains do not measure the triangular knight bonds");
  if (sampler == VP_SAMPLER_LEARNED_PLAQ && !L->net_ready)
    return fail(ctx, VP_ERR_ARG, "the learned sampler needs proposal weights (vp_proposal_set_weights)");
  if (sampler == VP_SAMPLER_LEARNED_PLAQ && (L->p.Ly < 2 || L->p.Lx < 2))
    return fail(ctx, VP_ERR_SHAPE, "plaquettes need Ly, Lx >= 2");
  L->sampler = sampler;
  return VP_OK;
}

vp_status vp_move_counts(vp_ctx* ctx, int32_t lat, int64_t* counts_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !counts_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  const int n = L->p.n_chains;
  hipStream_t s = ctx->stream;
  HIP_TRY(ctx, hipMemcpy2DAsync(counts_dev, 4 * sizeof(int64_t), (const char*)L->meta + offsetof(ChainMeta, accepted),
                                sizeof(ChainMeta), 2 * sizeof(int64_t), n, hipMemcpyDeviceToDevice, s));
  HIP_TRY(ctx, hipMemcpy2DAsync(counts_dev + 2, 4 * sizeof(int64_t),
                                (const char*)L->meta + offsetof(ChainMeta, p_accepted), sizeof(ChainMeta),
                                2 * sizeof(int64_t), n, hipMemcpyDeviceToDevice, s));
  if (L->role == TWIN_COLUMNS) launch_add_counts(ctx->lats[L->col].meta, counts_dev, 4, n, s);  // the vertical moves
  HIP_TRY(ctx, hipGetLastError());
  return VP_OK;
}

vp_status vp_proposal_forward(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n, float* logits_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !spins_dev || !logits_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (!L->net_ready) return fail(ctx, VP_ERR_ARG, "the proposal network has no weights yet");
  if (n < 1) return fail(ctx, VP_ERR_ARG, "n must be >= 1");
  NetWork w;
  if (!w.alloc(*L, n, ctx->stream)) return fail(ctx, VP_ERR_OOM, "proposal workspace allocation failed");
  net_forward(L->d_net, spins_dev, n, L->p.Ly, L->p.Lx, w.work, logits_dev, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return VP_OK;
}

vp_status vp_proposal_logits_sweep(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n, int32_t flip,
                                   double* logits_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !spins_dev || !logits_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (!L->net_ready) return fail(ctx, VP_ERR_ARG, "the proposal network has no weights yet");
  if (n < 1 || (flip != 0 && flip != 1)) return fail(ctx, VP_ERR_ARG, "n must be >= 1 and flip 0 or 1");
  if (L->p.Ly < 2 || L->p.Lx < 2) return fail(ctx, VP_ERR_SHAPE, "the lattice has no plaquettes");
  const int kind = L->p.prec == VP_BF16 ? 2 : (works_f64(L->p.prec) ? 1 : 0);
  net_local_logits(kind, L->d_net, L->d_net64, L->d_netbf, spins_dev, n, L->p.Ly, L->p.Lx, flip, logits_dev,
                   ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  return VP_OK;
}

vp_status vp_proposal_forward_noalloc(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n,
                                      float* logits_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !spins_dev || !logits_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (!L->net_ready) return fail(ctx, VP_ERR_ARG, "the proposal network has no weights yet");
  if (n < 1) return fail(ctx, VP_ERR_ARG, "n must be >= 1");
  const size_t need = net_forward_floats(n, L->p.Ly, L->p.Lx);
  if (need > NET_SCRATCH_FLOATS)
    return fail(ctx, VP_ERR_ARG, "n = %d needs %zu floats of scratch; the static scratch holds %zu (n <= %zu here)",
                n, need, NET_SCRATCH_FLOATS, NET_SCRATCH_FLOATS / net_forward_floats(1, L->p.Ly, L->p.Lx));
  int dev = 0;
  HIP_TRY(ctx, hipGetDevice(&dev));
  float* scratch = net_scratch_ptr(dev);
  if (!scratch) return fail(ctx, VP_ERR_DEVICE, "no static scratch on device %d (create the context there)", dev);
  net_forward(L->d_net, spins_dev, n, L->p.Ly, L->p.Lx, scratch, logits_dev, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  return VP_OK;
}

vp_status vp_proposal_loss_grad(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, const double* ratios_dev,
                                int32_t n, float* grad_dev, double* loss_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !spins_dev || !ratios_dev || !grad_dev || !loss_dev)
    return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (!L->net_ready) return fail(ctx, VP_ERR_ARG, "the proposal network has no weights yet");
  if (n < 1) return fail(ctx, VP_ERR_ARG, "n must be >= 1");
  if (L->p.Ly < 2 || L->p.Lx < 2) return fail(ctx, VP_ERR_SHAPE, "plaquettes need Ly, Lx >= 2");
  NetWork w;
  if (!w.alloc(*L, n, ctx->stream)) return fail(ctx, VP_ERR_OOM, "proposal workspace allocation failed");
  hipStream_t s = ctx->stream;
  net_loss_grad(L->d_net, spins_dev, ratios_dev, n, L->p.Ly, L->p.Lx, w.work, w.part, w.cnt, w.scal, grad_dev, s);
  HIP_TRY(ctx, hipMemcpyAsync(loss_dev, w.scal, sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return VP_OK;
}

vp_status vp_proposal_train(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, const double* ratios_dev,
                            int64_t n, int32_t epochs, int32_t batch, double lr, uint64_t seed,
                            double* loss_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !spins_dev || !ratios_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (!L->net_ready) return fail(ctx, VP_ERR_ARG, "the proposal network has no weights yet");
  if (n < 1 || epochs < 1 || batch < 1 || !(lr > 0.0)) return fail(ctx, VP_ERR_ARG, "need n, epochs, batch >= 1, lr > 0");
  if (n > INT32_MAX) return fail(ctx, VP_ERR_ARG, "at most 2^31 - 1 training configurations");
  if (L->p.Ly < 2 || L->p.Lx < 2) return fail(ctx, VP_ERR_SHAPE, "plaquettes need Ly, Lx >= 2");
  const int nb = (int)std::min<int64_t>(batch, n);
  NetWork w;
  if (!w.alloc(*L, nb, ctx->stream)) return fail(ctx, VP_ERR_OOM, "proposal workspace allocation failed");
  hipStream_t s = ctx->stream;
  const int H = L->p.Ly, W = L->p.Lx;
  std::vector<int32_t> perm(n);
  std::vector<double> eloss(epochs, 0.0);
  std::vector<double> bl;
  uint64_t state = seed ^ 0x9E3779B97F4A7C15ull;
  auto next = [&]() {  // splitmix64 (Steele, Lea, Flood 2014) for the host-side shuffle
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i >= 1; --i) std::swap(perm[i], perm[next() % (uint64_t)(i + 1)]);
    const int64_t nbatch = n / nb;  // whole batches only; the remainder rotates with the shuffle
    bl.assign(nbatch, 0.0);
    for (int64_t bi = 0; bi < nbatch; ++bi) {
      HIP_TRY(ctx, hipMemcpyAsync(w.idx, perm.data() + bi * nb, sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
      net_gather(spins_dev, ratios_dev, w.idx, nb, H, W, w.sb, w.rb, s);
      net_loss_grad(L->d_net, w.sb, w.rb, nb, H, W, w.work, w.part, w.cnt, w.scal, w.grad, s);
      net_adam(L->d_net, w.grad, L->d_adam, L->d_adam + NET_NPARAM, (float)lr, (int)++L->adam_t, s);
      HIP_TRY(ctx, hipMemcpyAsync(&bl[bi], w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
      // the host index buffer is reused by the next batch
      HIP_TRY(ctx, hipStreamSynchronize(s));
    }
    double m = 0.0;
    for (double v : bl) m += v;
    eloss[ep] = nbatch ? m / nbatch : 0.0;
  }
  net_cast_f64(L->d_net, L->d_net64, s);
  net_pack_bf16(L->d_net, L->d_netbf, s);
  HIP_TRY(ctx, hipGetLastError());
  if (loss_dev)
    HIP_TRY(ctx, hipMemcpyAsync(loss_dev, eloss.data(), sizeof(double) * epochs, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return VP_OK;
}

vp_status vp_gradient(vp_ctx* ctx, int32_t lat, const double* e_loc_dev, const void* dlnpsi_dev,
                      const int8_t* spins_dev, int64_t n_samples, double* grad_dev, double* e_mean_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !e_loc_dev || !dlnpsi_dev || !spins_dev || !grad_dev || !e_mean_dev)
    return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (n_samples < 1) return fail(ctx, VP_ERR_ARG, "n_samples must be >= 1");
  if (works_f64(L->p.prec))
    launch_gradient<double>(L->d_offs, L->d_coff, L->d_sizes, L->N, L->Np, e_loc_dev, (const double*)dlnpsi_dev,
                            spins_dev, n_samples, grad_dev, e_mean_dev, nullptr, ctx->stream);
  else
    launch_gradient<float>(L->d_offs, L->d_coff, L->d_sizes, L->N, L->Np, e_loc_dev, (const float*)dlnpsi_dev,
                           spins_dev, n_samples, grad_dev, e_mean_dev, nullptr, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  return VP_OK;
}

vp_status vp_sr_update(vp_ctx* ctx, int32_t lat, const double* e_loc_dev, const void* dlnpsi_dev,
                       const int8_t* spins_dev, int64_t n_samples, double shift, double lr, double* delta_dev) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !e_loc_dev || !dlnpsi_dev || !spins_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null pointer");
  if (n_samples < 2) return fail(ctx, VP_ERR_ARG, "n_samples must be >= 2");
  if (!(shift >= 0.0)) return fail(ctx, VP_ERR_ARG, "shift must be >= 0");
  if (L->Np > 32768) return fail(ctx, VP_ERR_SHAPE, "the dense S matrix needs Np <= 32768 (Np = %lld)", (long long)L->Np);
  if (n_samples * L->Np >= (int64_t)1 << 31) return fail(ctx, VP_ERR_SHAPE, "n_samples * Np must stay below 2^31");
  // the factorisation workspace: kept by the lattice from the first call on
  const int64_t nd = sr_work_doubles(L->Np, n_samples);
  if (!grow(ctx->stream, L->sr_work, sizeof(double) * nd) || !grow(ctx->stream, L->sr_flag, sizeof(int)))
    return fail(ctx, VP_ERR_OOM, "SR workspace");
  double* work = (double*)L->sr_work.p;
  int* flag = (int*)L->sr_flag.p;
  HIP_TRY(ctx, hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
  int rc = works_f64(L->p.prec)
               ? launch_sr<double>(L->d_offs, L->d_coff, L->d_sizes, L->N, L->Np, e_loc_dev, (const double*)dlnpsi_dev,
                                   spins_dev, n_samples, shift, lr, L->T, delta_dev, work, flag, ctx->stream)
               : launch_sr<float>(L->d_offs, L->d_coff, L->d_sizes, L->N, L->Np, e_loc_dev, (const float*)dlnpsi_dev,
                                  spins_dev, n_samples, shift, lr, L->T, delta_dev, work, flag, ctx->stream);
  int hflag = 0;
  hipError_t e1 = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  hipError_t e2 = hipStreamSynchronize(ctx->stream);
  if (rc != 0 || e1 != hipSuccess || e2 != hipSuccess) return fail(ctx, VP_ERR_DEVICE, "SR kernels failed");
  if (hflag) return fail(ctx, VP_ERR_NONFINITE, "S + shift I is not numerically positive definite");
  return stage_tensors(ctx, *L);
}

vp_status vp_sign_sgd_update(vp_ctx* ctx, int32_t lat, const double* grad_dev, double step_len, uint64_t step) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !grad_dev) return fail(ctx, VP_ERR_ARG, "bad lattice index or null gradient");
  launch_sign_sgd(L->T, grad_dev, L->Np, step_len, ctx->seed, lat, step, ctx->stream);
  HIP_TRY(ctx, hipGetLastError());
  return stage_tensors(ctx, *L);
}

vp_status vp_optimize(vp_ctx* ctx, int32_t lat, int32_t n_steps, int32_t n_burn, int32_t n_meas,
                      const double* delta_host, uint64_t step0, double* e_mean_host) {
  Lattice* L = get_lat(ctx, lat);
  if (!L || !delta_host) return fail(ctx, VP_ERR_ARG, "bad lattice index or null step lengths");
  if (n_steps < 0 || n_burn < 0 || n_meas < 1)
    return fail(ctx, VP_ERR_ARG, "need n_steps >= 0, n_burn >= 0, n_meas >= 1");
  const int64_t n = (int64_t)L->p.n_chains * n_meas;
  const size_t wsz = type_size(L->p.prec);
  // the samples of one step, the gradient and the mean energy: kept by the lattice
  hipStream_t s = ctx->stream;
  if (!grow(s, L->opt_lp, sizeof(double) * n) || !grow(s, L->opt_el, sizeof(double) * n) ||
      !grow(s, L->opt_grad, sizeof(double) * L->Np) || !grow(s, L->opt_em, sizeof(double)) ||
      !grow(s, L->opt_sg, n) || !grow(s, L->opt_so, n * L->N) || !grow(s, L->opt_dl, wsz * n * (L->Np / 2)))
    return fail(ctx, VP_ERR_OOM, "optimisation buffers");
  double* lp = (double*)L->opt_lp.p;
  double* el = (double*)L->opt_el.p;
  double* grad = (double*)L->opt_grad.p;
  double* em = (double*)L->opt_em.p;
  int8_t* sg = (int8_t*)L->opt_sg.p;
  int8_t* so = (int8_t*)L->opt_so.p;
  void* dl = L->opt_dl.p;
  vp_status st = VP_OK;
  for (int i = 0; i < n_steps && st == VP_OK; ++i) {
    // Algorithm 1: sample, Eq. (5) gradient, Eq. (10) update
    st = vp_sample(ctx, lat, n_burn, n_meas, lp, sg, el, dl, so, nullptr);
    // a chain that met a zero or non-finite amplitude left its rows unmeasured:
    // stop before they enter the gradient and the tensors
    if (st == VP_OK) st = check_flags(ctx, *L);
    if (st == VP_OK) st = vp_gradient(ctx, lat, el, dl, so, n, grad, em);
    if (st == VP_OK && e_mean_host) {
      if (hipMemcpyAsync(e_mean_host + i, em, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        st = fail(ctx, VP_ERR_DEVICE, "reading the step energy failed");
    }
    if (st == VP_OK) st = vp_sign_sgd_update(ctx, lat, grad, delta_host[i], step0 + (uint64_t)i);
  }
  hipStreamSynchronize(s);
  return st;
}

vp_status vp_stats_tau(const double* x, int32_t n_chains, int32_t len, double c, double* tau, double* mean_out,
                       double* stderr_out) {
  if (!x || !tau || !mean_out || !stderr_out || n_chains < 1 || len < 2 || !(c > 0))
    return fail(nullptr, VP_ERR_ARG, "bad arguments to vp_stats_tau");
  double total = 0.0, var_mean = 0.0;
  std::vector<double> d(len);
  for (int ch = 0; ch < n_chains; ++ch) {
    const double* s = x + (int64_t)ch * len;
    double m = 0.0;
    for (int t = 0; t < len; ++t) m += s[t];
    m /= len;
    total += m;
    for (int t = 0; t < len; ++t) d[t] = s[t] - m;
    double c0 = 0.0;
    for (int t = 0; t < len; ++t) c0 += d[t] * d[t];
    c0 /= len;
    double tau_c = 0.5;
    if (c0 > 0.0) {
      for (int M = 1; M < len; ++M) {
        double cm = 0.0;
        for (int t = 0; t + M < len; ++t) cm += d[t] * d[t + M];
        tau_c += cm / len / c0;
        if (M >= c * tau_c) break;
      }
    }
    tau[ch] = tau_c;
    var_mean += c0 * 2.0 * tau_c / len;
  }
  *mean_out = total / n_chains;
  *stderr_out = std::sqrt(std::max(var_mean, 0.0)) / n_chains;
  return VP_OK;
}

vp_status vp_timing_enable(vp_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(nullptr, VP_ERR_ARG, "null context");
  fold_timing(ctx);
  for (int i = 0; i < VP_NPHASE; ++i) { ctx->ph_ms[i] = 0.0; ctx->ph_n[i] = 0; }
  ctx->timing = enable != 0;
  return VP_OK;
}

vp_status vp_timing_read(vp_ctx* ctx, double* ms_host, int64_t* launches_host) {
  if (!ctx || !ms_host || !launches_host) return fail(ctx, VP_ERR_ARG, "null argument");
  fold_timing(ctx);
  for (int i = 0; i < VP_NPHASE; ++i) { ms_host[i] = ctx->ph_ms[i]; launches_host[i] = ctx->ph_n[i]; }
  return VP_OK;
}

vp_status vp_sync(vp_ctx* ctx) {
  if (!ctx) return fail(nullptr, VP_ERR_ARG, "null context");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < ctx->n_user; ++i) {  // a transposed lattice is checked with its own
    Lattice& L = ctx->lats[i];
    if (!L.chains_ready) continue;
    vp_status st = check_flags(ctx, L);
    if (st != VP_OK) return st;
  }
  return VP_OK;
}

}  // extern "C"
