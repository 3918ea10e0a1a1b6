/*
 * vmcpeps.h -- C ABI of the MI355X (gfx950) library for variational Monte Carlo
 * on finite open-boundary PEPS (Liu, Huang, Gong, Gu, "Accurate simulation
 * for finite projected entangled pair states in two dimensions").
 *
 * The calls follow the statement of the method in Sec. II.A-B and Alg. 1 of
 * the paper: initialise tensors, generate configurations by sequential
 * bond-visiting Metropolis sweeps (generateConfiguration), contract the
 * single-layer network for Psi(S) (contractNetwork), evaluate E_loc from pair
 * ratios Psi(S')/Psi(S) and the log-derivatives G = dlnPsi/dA from defect
 * networks (contractDefectNetwork), then form the gradient and update.
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice: Ly x Lx open-boundary square lattice, sites (y, x), y = 0 top row,
 *   k = y*Lx + x.  Spins are int8 0/1 (0 is S^z = +1/2), S^z_tot = 0 sector.
 * Tensors (Sec. II.A Eq. (1)): site k holds T_k[s][l][u][r][d]; legs on the
 *   open boundary have dimension 1, bulk legs dimension D.  The "canonical
 *   flat" parameter vector is the concatenation over k of these blocks, length
 *   Np = vp_num_params(); float64.
 * Log-derivatives (Sec. II.A Eqs. (6)-(7)): per sample, the "compact" vector
 *   of length Np/2 holds, for every site k in order, the l*u*r*d derivatives
 *   of the occupied slot s_k (the other slot is zero by construction).
 * Hamiltonian (Sec. II.A Eq. (3), App. C Eq. (Elocal)):
 *   H = J1 sum_NN S_i.S_j + J2 sum_diag S_i.S_j, S = sigma/2.
 *   VP_GEOM_TRIANGULAR (Sec. III.B, Fig. 7(a): the triangular lattice drawn
 *   on the square grid): the diagonal (y,x)-(y+1,x+1) of every plaquette is a
 *   nearest-neighbour bond (coupling J1); the next-nearest neighbours
 *   (coupling J2) are the other diagonal (y,x+1)-(y+1,x) and the knight bonds
 *   (y,x)-(y+1,x+2) (a 2-row network over three columns) and (y,x)-(y+2,x+1)
 *   (the same bond of the transposed lattice, site (y,x) -> (x,y): the
 *   context keeps that lattice beside the caller's, counted by
 *   vp_workspace_bytes, and evaluates it for every measured configuration).
 *   With J2 != 0 the triangular lattice is measured with the per-phase
 *   schedule and the pair or learned samplers (VP_ERR_UNSUPPORTED otherwise),
 *   and the simple update evolves its diagonals but not its knight bonds.
 * Pair order (the "ratios" outputs): horizontal bonds row by row, then
 *   vertical bonds row by row, then for every plaquette (y, x) the two
 *   diagonals (y,x)-(y+1,x+1) and (y,x+1)-(y+1,x) when a diagonal is coupled
 *   (J2 != 0, or the triangular geometry), then (triangular, J2 != 0) the
 *   bonds (y,x)-(y+1,x+2) for y < Ly-1, x < Lx-2 and (y,x)-(y+2,x+1) for
 *   y < Ly-2, x < Lx-1, row-major; an uncoupled bond's ratio is 0.
 * Contraction (App. B, App. C): boundary MPS truncated to Dc by the canonical
 *   SVD compression (left-to-right orthogonalisation, right-to-left truncation
 *   keeping the Dc largest singular values); 3-line row networks for
 *   horizontal pairs and 2-row (4-line) networks for vertical and diagonal
 *   pairs; every ratio divides by the same network with the current tensors.
 * Precision (vp_lattice.prec): VP_FP64 contracts in float64; VP_FP32 in
 *   float32 on MFMA; VP_BF16 stores tensors, boundaries and environments in
 *   float64, takes the 2-row steps of the sampling pass (the ratios that decide
 *   Metropolis moves) with bf16 operands and float32 accumulation (its 3-line
 *   steps run in float64 where a fused float64 step is built, D = 8 and
 *   Dc = 16, which is faster there), and measures Psi, E_loc and G in float64
 *   (App. D: a ratio error of a few bf16 ulps changes acceptance
 *   probabilities by as much, which the chain tolerates; the estimators are
 *   not protected by that argument, and float32 measurements of strongly
 *   cancelling networks miss the 1e-4 per-site energy tolerance).  Every mode
 *   keeps an exact power-of-two scale per network column, accumulates
 *   log|Psi| and normalises ratios in float64, and compresses boundaries in
 *   float64.  The "working precision" below is float32 for VP_FP32 and
 *   float64 otherwise.
 * Randomness: Philox4x64-10 (Salmon et al., SC'11) under key (seed, lattice);
 *   Metropolis uniforms use counter (chain, sweep, bond, 4), where bond counts
 *   the visits of one sweep: row y's horizontal bonds, then the vertical bonds
 *   between rows y and y+1, for y = 0, 1, ...
 *
 * Memory: every pointer argument named *_dev is a device pointer owned by the
 *   caller (for example a torch tensor's data_ptr on the same device);
 *   pointers named *_host are host pointers.  The library owns only its
 *   internal workspace: what the sweeps and vp_eval_sis need is allocated by
 *   vp_create; the workspaces of vp_sr_update, vp_optimize, vp_simple_update
 *   and the proposal network calls depend on their arguments, are allocated by the first call
 *   that needs them and kept for later calls (replaced by a larger one when a
 *   call needs more).  vp_destroy frees all of it.
 * Streams: work is enqueued on the hipStream_t given to vp_create (NULL = the
 *   null stream).  Calls return once the work is enqueued unless stated
 *   otherwise; vp_sync waits and reports device-side error flags.
 * Errors: every call returns a vp_status; vp_last_error(ctx) returns the
 *   message of the last failure on that context.  No outputs are promised
 *   after an error.  A context is not thread-safe; distinct contexts are
 *   independent.
 */
#ifndef VMCPEPS_H
#define VMCPEPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VP_OK = 0,
  VP_ERR_ARG = 1,            /* null pointer, index out of range, bad enum */
  VP_ERR_SHAPE = 2,          /* D < 1, Dc < 1, odd N, spins not in S^z = 0, sizes too large */
  VP_ERR_OOM = 3,            /* device allocation failed */
  VP_ERR_DEVICE = 4,         /* a HIP runtime call failed */
  VP_ERR_ZERO_AMPLITUDE = 5, /* a network that must be non-zero was exactly zero */
  VP_ERR_NONFINITE = 6,      /* a non-finite value appeared in a network */
  VP_ERR_UNSUPPORTED = 7     /* the requested mode is not built */
} vp_status;

typedef enum { VP_FP64 = 0, VP_FP32 = 1, VP_BF16 = 2 } vp_prec;

/* Samplers (vp_set_sampler).  VP_SAMPLER_PAIR_SEQ: the sequential
 * nearest-neighbour exchange sweep of Sec. II.A Eq. (9).
 * VP_SAMPLER_LEARNED_PLAQ: the same sweep with a learned plaquette move after
 * each vertical bond (see vp_set_sampler).  VP_SAMPLER_SIS_PAIR: chains of the
 * weight |Phi(S)|^2 of the spin-inversion symmetrised amplitude (Sec. II.B;
 * see vp_set_sampler). */
typedef enum { VP_SAMPLER_PAIR_SEQ = 0, VP_SAMPLER_LEARNED_PLAQ = 1, VP_SAMPLER_SIS_PAIR = 2 } vp_sampler;

/* Boundary truncation to Dc (App. B).  VP_COMPRESS_CANONICAL: the canonical
 * SVD compression (left-to-right orthogonalisation, right-to-left truncation
 * keeping the Dc largest singular values; float64 in every precision).
 * VP_COMPRESS_VARIATIONAL: the paper's variational fit, minimising
 * ||M_y|U_{y-1}> - |U_y>||^2 by fit_sweeps sweeps of single-site updates (in
 * the working precision): start from the leading k_l x k_r blocks of the
 * product sites (right-orthonormal form, state kept), then per sweep each site
 * replaced by the Q of the optimal site's QR (left to right) and by the
 * orthonormal rows of its LQ (right to left); the optimal site 0 carries the
 * norm.  Both use the same bond dimensions.  Sizes: D <= 16 and Dc <= 64;
 * D*Dc <= 128 for the canonical compression (its eigenproblems), D*Dc <= 192
 * for the fit (Dc = 3D at D = 8, the measuring cutoff of Sec. II.A and App. D).
 * The persistent schedule
 * (VP_SCHED_PERSISTENT, vp_sample_batch) runs the canonical compression only:
 * with VP_COMPRESS_VARIATIONAL it returns VP_ERR_UNSUPPORTED, and vp_autotune
 * skips it (its time reads -1). */
typedef enum { VP_COMPRESS_CANONICAL = 0, VP_COMPRESS_VARIATIONAL = 1 } vp_compress;

/* Lattice geometry of the Hamiltonian (see "Hamiltonian" above); the PEPS is
 * the square-lattice one in both. */
typedef enum { VP_GEOM_SQUARE = 0, VP_GEOM_TRIANGULAR = 1 } vp_geometry;

/* How the vertical bonds' ratios are contracted (App. C: the horizontal terms
 * of row k from 3-line networks between its row boundaries, the other terms
 * "similarly computed").  VP_VERT_ROWPAIR: the 2-row network of rows y, y+1
 * between U_{y-1} and D_{y+2}.  VP_VERT_COLUMN: column-wise boundaries - the
 * vertical bond (y,x)-(y+1,x) is the horizontal bond (x,y)-(x,y+1) of the
 * transposed lattice (site (y,x) -> (x,y), legs (l,u,r,d) -> (u,l,d,r); the
 * same state), whose 3-line networks run between column boundary MPS.  The
 * context keeps that transposed lattice beside the user's (its workspace is
 * counted by vp_workspace_bytes) and refreshes its tensors whenever the
 * tensors change.  A sweep of vp_sample then visits the horizontal bonds row
 * by row (row boundaries, bond indices as in VP_VERT_ROWPAIR), then the
 * vertical bonds column by column: the transposed lattice's horizontal pass,
 * after a lower-boundary pass of its own, with Philox key word 1 = lattice
 * index + 65536 and bond index x(2Ly-1)+y for the bond (y,x)-(y+1,x).  A
 * measured sweep evaluates the final configuration (Psi and G from the row
 * networks, E_loc from both).  Nearest-neighbour square lattices only
 * (J2 = 0), the pair sampler and the per-phase schedule
 * (VP_ERR_UNSUPPORTED otherwise). */
typedef enum { VP_VERT_ROWPAIR = 0, VP_VERT_COLUMN = 1 } vp_vertical;

typedef struct {
  int32_t Ly, Lx;      /* lattice extent */
  int32_t D;           /* PEPS virtual bond dimension */
  int32_t Dc;          /* boundary-MPS cutoff */
  double J1, J2;       /* nearest-neighbour and diagonal couplings */
  int32_t prec;        /* vp_prec of the contractions */
  int32_t n_chains;    /* Markov chains kept on the device */
  int32_t compress;    /* vp_compress (0 = canonical, the zero-initialised default) */
  int32_t fit_sweeps;  /* sweeps of VP_COMPRESS_VARIATIONAL (0..64) */
  int32_t geometry;    /* vp_geometry (0 = square, the zero-initialised default) */
  int32_t vertical;    /* vp_vertical (0 = 2-row networks, the default) */
} vp_lattice;

typedef struct vp_ctx vp_ctx;

/* Create a context for n_lats lattices; allocates every device buffer the
 * sweeps need for n_chains chains of each lattice.  seed is the Philox key
 * word 0; the lattice index is key word 1.  stream: a hipStream_t or NULL. */
vp_status vp_create(const vp_lattice* lats, int32_t n_lats, uint64_t seed, void* stream, vp_ctx** out);
vp_status vp_destroy(vp_ctx* ctx);
const char* vp_last_error(const vp_ctx* ctx);

/* Np = sum_k 2*dim(l)dim(u)dim(r)dim(d) (Sec. II.B counts 7,496,192 for 32x32, D=8). */
int64_t vp_num_params(const vp_lattice* lat);
/* Bytes of device workspace vp_create allocates for this lattice. */
int64_t vp_workspace_bytes(const vp_lattice* lat);

/* Canonical flat float64 tensors in or out (Np numbers).  T_dev is a device pointer. */
vp_status vp_set_tensors(vp_ctx* ctx, int32_t lat, const double* T_dev);
vp_status vp_get_tensors(vp_ctx* ctx, int32_t lat, double* T_dev);
/* T = scale * xi + perturb * xi', xi, xi' ~ N(0,1) by Box-Muller on Philox
 * words 0 and 1 of counters (p, 0, 0, 1) and (p, 0, 0, 2), key (seed, lat).
 * scale <= 0 selects 1/D^2. */
vp_status vp_init_tensors(vp_ctx* ctx, int32_t lat, uint64_t seed, double scale, double perturb);

/* Set every chain's configuration: spins_dev [n_chains][N] int8, or NULL for
 * a Fisher-Yates shuffle of the Neel list per chain (index j = floor(u (i+1))
 * from counter (chain, 0, i, 3)).  Resets the sweep counters to 0. */
vp_status vp_init_chains(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev);

/* Run n_burn + n_meas sequential sweeps on every chain (Sec. II.A Eq. (9)),
 * measuring after each of the last n_meas.  Outputs, indexed [chain][m]:
 * log_abs_psi_dev, sign_dev (+1/-1), e_loc_dev (total energy, not per site),
 * dlnpsi_dev ([chain][m][Np/2] in the working precision: float32 for VP_FP32,
 * float64 otherwise; may be NULL), spins_out_dev ([chain][m][N], may be NULL).
 * accept_dev ([chain][2] int64: accepted, proposed; accumulated; may be NULL). */
vp_status vp_sample(vp_ctx* ctx, int32_t lat, int32_t n_burn, int32_t n_meas,
                    double* log_abs_psi_dev, int8_t* sign_dev, double* e_loc_dev,
                    void* dlnpsi_dev, int8_t* spins_out_dev, int64_t* accept_dev);

/* Launch schedules of a lattice's sweeps (vp_set_schedule).
 * VP_SCHED_PHASES: one launch per phase and row, every chain in each.
 * VP_SCHED_PERSISTENT: one launch per sweep; its work-groups take chains from
 *   a queue and run each chain's whole sweep (all rows, both passes).
 * VP_SCHED_GRAPH: the per-phase launches of one sweep are captured once per
 *   vp_sample call into a HIP graph and replayed every sweep.
 * All three produce the same results (float64: bit-identical chains); phase
 * timing (vp_timing_*) then books whole sweeps under VP_PH_OTHER. */
typedef enum { VP_SCHED_PHASES = 0, VP_SCHED_PERSISTENT = 1, VP_SCHED_GRAPH = 2 } vp_schedule;
vp_status vp_set_schedule(vp_ctx* ctx, int32_t lat, int32_t schedule);

/* Outputs of one lattice in vp_sample_batch (device pointers, same layout as
 * vp_sample's; dlnpsi_dev and spins_out_dev may be NULL). */
typedef struct {
  double* log_abs_psi_dev;
  int8_t* sign_dev;
  double* e_loc_dev;
  void* dlnpsi_dev;
  int8_t* spins_out_dev;
} vp_outputs;

/* vp_sample for several lattices of one context at once (uneven sizes and
 * couplings allowed; D, Dc and precision must be equal): each sweep is one
 * persistent launch whose queue holds every chain of every listed lattice,
 * largest lattices first.  lats_host [n_lats] lattice indices (distinct);
 * outs_host [n_lats] (may be NULL when n_meas = 0).  Each lattice keeps its
 * own sampler. */
vp_status vp_sample_batch(vp_ctx* ctx, int32_t n_lats, const int32_t* lats_host, int32_t n_burn, int32_t n_meas,
                          const vp_outputs* outs_host);

/* Times `sweeps` unmeasured sweeps of the lattice under each schedule (after
 * one warm-up sweep each; the chains advance by 3 (sweeps + 1) sweeps, which
 * count as burn-in), keeps the fastest and returns it in *schedule_out;
 * ms_host [3] (may be NULL) receives the milliseconds per sweep of
 * VP_SCHED_PHASES, VP_SCHED_PERSISTENT and VP_SCHED_GRAPH, -1 for a schedule
 * the lattice cannot run (the persistent one with the variational fit; both
 * others with VP_VERT_COLUMN, the triangular knight bonds or the |Phi|^2
 * chains).  Waits. */
vp_status vp_autotune(vp_ctx* ctx, int32_t lat, int32_t sweeps, double* ms_host, int32_t* schedule_out);

/* Tile variants of the fused float32 / float64 2-row column step (App. C: the
 * 4-line environment step, used by the vertical sweep, the right 2-row
 * environments and the 2-row measurement) at D = 8, Dc = 16: the step
 * contracts the upper-boundary index b in blocks of BB, VP_TILE_DEFAULT
 * BB = Dc/4, VP_TILE_SMALL Dc/8, VP_TILE_LARGE Dc/2 (a larger block needs more
 * LDS per work-group, a smaller one more barriers per step).  The blocking
 * only partitions the output, so every variant gives bit-identical results;
 * other shapes and the bf16 sampling steps have one variant, and the
 * persistent schedule always takes the default.  vp_set_tile selects one for
 * a lattice (VP_ERR_ARG for an unknown variant). */
typedef enum { VP_TILE_DEFAULT = 0, VP_TILE_SMALL = 1, VP_TILE_LARGE = 2, VP_N_TILES = 3 } vp_tile;
vp_status vp_set_tile(vp_ctx* ctx, int32_t lat, int32_t tile);

/* The tile autotuner: times `sweeps` unmeasured sweeps of the lattice under
 * each tile variant with its current schedule (after one warm-up sweep each;
 * the chains advance by VP_N_TILES (sweeps + 1) sweeps, which count as
 * burn-in), keeps the fastest and returns it in *tile_out; ms_host
 * [VP_N_TILES] (may be NULL) receives the milliseconds per sweep of each.
 * Waits. */
vp_status vp_autotune_tiles(vp_ctx* ctx, int32_t lat, int32_t sweeps, double* ms_host, int32_t* tile_out);

/* Record the sampler's decisions: while trace_dev is set (NULL clears it),
 * every sweep of vp_sample overwrites trace_dev[chain][b][0..1] with the ratio
 * rho = Psi(S')/Psi(S) that bond b's Metropolis test used (float64, after the
 * exact power-of-two rescaling) and 1.0 if the exchange was accepted, 0.0
 * otherwise; b = y(2Lx-1)+x for the horizontal bond (y,x)-(y,x+1) and
 * y(2Lx-1)+(Lx-1)+x for the vertical bond (y,x)-(y+1,x); pairs that are
 * parallel when visited get (0, 0).  trace_dev holds n_chains * n_bonds * 2
 * float64 with n_bonds = Ly(Lx-1) + (Ly-1)Lx, stays owned by the caller and
 * must outlive its use. */
vp_status vp_trace_ratios(vp_ctx* ctx, int32_t lat, double* trace_dev);

/* Evaluate fixed configurations spins_dev [n_cfg][N] (n_cfg <= n_chains):
 * the same outputs as one measured sweep without Metropolis moves, plus every
 * pair ratio (ratios_dev [n_cfg][n_pairs], 0 for parallel pairs; may be NULL).
 * n_pairs = Ly(Lx-1) + (Ly-1)Lx (+ 2(Ly-1)(Lx-1) when a diagonal is coupled:
 * J2 != 0 or VP_GEOM_TRIANGULAR; + (Ly-1)(Lx-2) + (Ly-2)(Lx-1) for the knight
 * bonds of VP_GEOM_TRIANGULAR with J2 != 0). */
vp_status vp_eval(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n_cfg,
                  double* log_abs_psi_dev, int8_t* sign_dev, double* e_loc_dev,
                  void* dlnpsi_dev, double* ratios_dev);

/* Spin-inversion symmetrisation (Sec. II.B, symmetrised wave function
 * Phi(S) = Psi(S) + Psi(Sbar), Sbar = S with every spin reversed; observables
 * are taken with the weight |Phi(S)|^2).  For the configurations spins_dev
 * [n_cfg][N] (1 <= n_cfg <= n_chains, S^z_tot = 0) evaluates S and Sbar as
 * vp_eval does and writes, per configuration (device pointers, n_cfg entries
 * each, caller-owned): log_abs_phi_dev log|Phi(S)|, sign_phi_dev its sign,
 * e_loc_phi_dev E_Phi(S) = sum_S' <S|H|S'> Phi(S')/Phi(S)
 * = (Psi(S) E_loc(S) + Psi(Sbar) E_loc(Sbar)) / Phi(S), and log_w_dev
 * log(|Phi(S)|^2 / |Psi(S)|^2), the weight that turns samples of |Psi|^2 (from
 * vp_sample) into samples of |Phi|^2: <O>_Phi = sum w O / sum w.  Where
 * Psi(Sbar) = -Psi(S) exactly, log|Phi| and log w are -inf, the sign 0 and
 * E_Phi 0.  Uses the n_chains (N + 17) bytes of scratch reserved by vp_create;
 * waits for the stream; same preconditions and errors as vp_eval; invalidates
 * the sampler's state. */
vp_status vp_eval_sis(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n_cfg,
                      double* log_abs_phi_dev, int8_t* sign_phi_dev, double* e_loc_phi_dev, double* log_w_dev);

/* Two truncation cutoffs (Sec. II.A, App. D): the chains of lattice
 * lat_sample move with its cutoff Dc1 (a ratio only meets a uniform number,
 * so a modest cutoff suffices), and after every sweep past the n_burn first
 * their configurations are measured on lattice lat_measure with its cutoff
 * Dc2, as vp_eval does.  The two lattices must agree in Ly, Lx, D, J1, J2 and
 * precision; lat_measure needs at least as many chains and its tensors set
 * (normally the same as lat_sample's); its chain slots are overwritten.
 * Outputs as in vp_sample (row chain * n_meas + m; spins_out_dev and
 * dlnpsi_dev may be NULL).  The sampling chains' state advances exactly as
 * under vp_sample. */
vp_status vp_sample_split(vp_ctx* ctx, int32_t lat_sample, int32_t lat_measure, int32_t n_burn, int32_t n_meas,
                          double* log_abs_psi_dev, int8_t* sign_dev, double* e_loc_dev, void* dlnpsi_dev,
                          int8_t* spins_out_dev);

/* Psi(S')/Psi(S) for the flip of all four spins of every plaquette (y, x)
 * (sites (y,x), (y,x+1), (y+1,x), (y+1,x+1)) that holds two up and two down
 * spins; ratios_dev [n_cfg][(Ly-1)(Lx-1)] float64, 0 for the other plaquettes.
 * Each ratio is the two-row network of rows y, y+1 with columns x and x+1
 * exchanged, divided by the same network with the current tensors (the
 * construction App. C uses for vertical pairs).  Same preconditions and
 * synchronous error reporting as vp_eval; invalidates the sampler's state. */
vp_status vp_plaquette_ratios(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n_cfg,
                              double* ratios_dev);

/* ---- learned plaquette proposal (not in the paper) ------------------------
 * Network f(S): spins as +1 (s = 0) / -1 (s = 1) in one channel;
 * conv3x3(1->32), ReLU, conv3x3(32->32), ReLU, conv3x3(32->32), ReLU,
 * conv3x3(32->1), zero padding at the open boundary,
 * out[co][y][x] = b[co] + sum W[co][ci][ky][kx] in[ci][y+ky-1][x+kx-1].
 * The logit of plaquette (y, x) is the output at (y, x); its propensity is
 * pi = sigmoid(logit).  Parameters: float32, flat, in the order
 * W1[32][1][3][3] b1[32] W2[32][32][3][3] b2[32] W3[32][32][3][3] b3[32]
 * W4[1][32][3][3] b4[1] (vp_proposal_num_params() = 19105 numbers). */
int64_t vp_proposal_num_params(void);
/* Copy the parameters in (device pointer); resets the optimiser state. */
vp_status vp_proposal_set_weights(vp_ctx* ctx, int32_t lat, const float* w_dev);
vp_status vp_proposal_get_weights(vp_ctx* ctx, int32_t lat, float* w_dev);
/* Logit maps of n configurations: logits_dev [n][Ly][Lx] float32.  Waits. */
vp_status vp_proposal_forward(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n, float* logits_dev);
/* The logits of every plaquette (y, x) of n configurations as the learned
 * sweep evaluates them inside the sampler: logits_dev [n][(Ly-1)(Lx-1)]
 * float64, plaquette index y (Lx-1) + x (all plaquettes, movable or not),
 * from the local 9x9 window of each; with flip = 1 the plaquette's four spins
 * are flipped first (the reverse proposal).  VP_FP64 and VP_FP32 evaluate in
 * the working precision; VP_BF16 in bf16 inference: weights and ReLU outputs
 * rounded to bf16 (nearest, ties to even), float32 accumulation on the bf16
 * MFMA, biases in float32.  Asynchronous; VP_ERR_SHAPE for a lattice of one
 * row or column. */
vp_status vp_proposal_logits_sweep(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n, int32_t flip,
                                   double* logits_dev);
/* vp_proposal_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and the same logits, bit for bit, with the
 * activations in a fixed 16 MiB array of device memory per GPU (looked up once
 * per device by vp_create) instead of the lattice's workspace.  Calls no
 * allocation routine and does not wait: the call only enqueues on the
 * context's stream.  n * Ly * Lx * 97 floats must fit the 4 Mi floats of that
 * array (n <= 168 at 16x16, n <= 42 at 32x32), otherwise VP_ERR_ARG and nothing
 * is launched.  Nothing in the array needs clearing (every activation is
 * written before it is read), but every call on one GPU shares it: calls that
 * overlap on one GPU (other streams, other contexts, other threads) race. */
vp_status vp_proposal_forward_noalloc(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, int32_t n,
                                      float* logits_dev);
/* Training loss and its gradient on n configurations: the mean over all
 * movable plaquettes of the binary cross-entropy of pi against the acceptance
 * probability a = min(1, rho^2), rho from ratios_dev (as written by
 * vp_plaquette_ratios).  grad_dev [vp_proposal_num_params()] float32,
 * loss_dev one float64.  Waits. */
vp_status vp_proposal_loss_grad(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, const double* ratios_dev,
                                int32_t n, float* grad_dev, double* loss_dev);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) on that loss over
 * epochs passes of shuffled minibatches of `batch` configurations (whole
 * batches only; the shuffle is seeded by seed).  loss_dev [epochs] float64
 * (mean minibatch loss per epoch) may be NULL.  Keeps its workspace (sized by
 * the batch) for later calls; waits. */
vp_status vp_proposal_train(vp_ctx* ctx, int32_t lat, const int8_t* spins_dev, const double* ratios_dev,
                            int64_t n, int32_t epochs, int32_t batch, double lr, uint64_t seed,
                            double* loss_dev);
/* Select the sampler of the following vp_sample calls.
 * VP_SAMPLER_LEARNED_PLAQ (needs weights): within the row-pair step of every
 * row y < Ly-1, right after the vertical bond (y,x)-(y+1,x), x < Lx-1, a
 * plaquette (y, x) holding two up and two down spins is proposed with
 * probability pi(S) (Philox word 0 of counter (chain, sweep, y(Lx-1)+x, 6))
 * and its flip accepted iff u < rho^2 pi(S')/pi(S), u = word 1 of the same
 * counter: Metropolis-Hastings for a propose-or-stay move, so |Psi|^2 stays
 * the stationary distribution whatever the weights.  The network runs in the
 * working precision.
 * VP_SAMPLER_SIS_PAIR (n_chains even, the per-phase schedule): Markov chains
 * of |Phi(S)|^2, Phi(S) = Psi(S) + Psi(Sbar), Sbar = S with every spin
 * reversed (Sec. II.B).  Chain c < n_chains/2 carries S and chain
 * c + n_chains/2 its reversal; every vp_sample call first sets the second half
 * to the reversal of the first, rebuilds the lower boundaries and contracts
 * both amplitudes top-down.  The pair visits the bonds in the Eq. (9) order;
 * each chain's ratio r = Psi(S')/Psi(S), rbar = Psi(Sbar')/Psi(Sbar) comes
 * from its own environments, and the exchange of the same pair in both is
 * accepted iff u < q^2, q = (Psi(S) r + Psi(Sbar) rbar) / (Psi(S) + Psi(Sbar)),
 * u from chain c's Philox counter (c, sweep, bond, 4); Psi(S) and Psi(Sbar)
 * are the last top-down contractions times the ratios of the moves accepted
 * since.  vp_sample then writes n_chains/2 samples per measured sweep, indexed
 * [c][m]: log|Phi|, sign(Phi), E_Phi(S) = (Psi(S) E_loc(S) + Psi(Sbar)
 * E_loc(Sbar)) / (Psi(S) + Psi(Sbar)) (the Heisenberg elements are invariant
 * under the reversal), and S; dlnpsi_dev must be NULL (not produced) and
 * accept_dev covers the first n_chains/2 chains.  An exactly zero Psi(S) or
 * Psi(Sbar) in a visited network flags the pair (VP_ERR_ZERO_AMPLITUDE).
 * vp_sample_batch and vp_sample_split return VP_ERR_UNSUPPORTED for it. */
vp_status vp_set_sampler(vp_ctx* ctx, int32_t lat, int32_t sampler);
/* Move counters since vp_init_chains: counts_dev [n_chains][4] int64 =
 * (pair accepted, pair proposed, plaquette accepted, plaquette proposed). */
vp_status vp_move_counts(vp_ctx* ctx, int32_t lat, int64_t* counts_dev);

/* Eq. (5): grad = <G E_loc> - <G><E_loc> over n_samples samples (compact
 * dlnpsi in the working precision, their spins [n][N]); grad_dev [Np] float64,
 * e_mean_dev one float64. */
vp_status vp_gradient(vp_ctx* ctx, int32_t lat, const double* e_loc_dev, const void* dlnpsi_dev,
                      const int8_t* spins_dev, int64_t n_samples, double* grad_dev, double* e_mean_dev);

/* Stochastic reconfiguration: (S + shift I) delta = g with S the covariance of
 * the full-layout log-derivatives and g the Eq. (5) gradient, solved in float64
 * by a blocked Cholesky factorisation on the device; then T <- T - lr * delta.
 * delta_dev [Np] may be NULL.  Needs Np <= 32768 and n_samples * Np < 2^31;
 * needs (8 Np^2 + 8 n_samples Np) bytes of workspace, kept by the lattice for
 * later calls, and waits for completion.  VP_ERR_NONFINITE if S + shift I is not numerically
 * positive definite. */
vp_status vp_sr_update(vp_ctx* ctx, int32_t lat, const double* e_loc_dev, const void* dlnpsi_dev,
                       const int8_t* spins_dev, int64_t n_samples, double shift, double lr,
                       double* delta_dev);

/* Eq. (10): T <- T - r * step_len * sgn(grad), r = uniform from counter
 * (p, step, 0, 5) per element p. */
vp_status vp_sign_sgd_update(vp_ctx* ctx, int32_t lat, const double* grad_dev, double step_len, uint64_t step);

/* Algorithm 1 for n_steps optimisation steps: each step runs vp_sample
 * (n_burn sweeps, then n_meas measured sweeps of every chain), the Eq. (5)
 * gradient over the n_chains * n_meas samples and the Eq. (10) update with
 * step length delta_host[i] and random counter step0 + i (Sec. II.B uses
 * 0.005, 0.002, 0.001 and 0.0005 in successive stages).  e_mean_host
 * [n_steps] (may be NULL) receives each step's mean E_loc, measured before
 * its update.  Keeps the buffers of one step's samples for later calls and
 * waits for completion.  Stops with VP_ERR_ZERO_AMPLITUDE or VP_ERR_NONFINITE,
 * before that step's gradient and update, when a chain met a zero or
 * non-finite amplitude (its rows were not measured); the tensors then hold the
 * previous step's update. */
vp_status vp_optimize(vp_ctx* ctx, int32_t lat, int32_t n_steps, int32_t n_burn, int32_t n_meas,
                      const double* delta_host, uint64_t step0, double* e_mean_host);

/* Simple-update imaginary-time evolution (App. A), the initialisation the
 * paper runs before Algorithm 1.  The PEPS is held as site tensors and a
 * diagonal lambda (D numbers) on every link; a step applies exp(-dt J1
 * S_i.S_j) once to every link, in four classes of links that share no site
 * (horizontal links with x even, x odd, vertical links with y even, y odd),
 * then, when J2 != 0, exp(-dt J2 S_i.S_j) to both diagonals of every
 * plaquette, in four classes of plaquettes (y mod 2, x mod 2), diagonals
 * before anti-diagonals.  Per link: the outer links' lambdas multiply both
 * tensors, each is reduced by a thin Householder QR, the gate acts on the
 * reduced two-site tensor (lambda of the link between), its truncated SVD
 * gives the new lambda (the leading D singular values above 1e-6 of the
 * largest, normalised to unit 2-norm) and the new tensors, from which the
 * outer lambdas are divided out again.  Per diagonal (Fig. 8): the pair is
 * joined through a corner site ((y,x)-(y+1,x+1) through (y,x+1),
 * (y,x+1)-(y+1,x) through (y,x)); the end tensors are QR-reduced, the gate
 * acts on the reduced three-site tensor, and two truncated SVDs give both
 * links' lambdas and the three new tensors.  The first call on the
 * current tensors starts from them with every lambda 1; a later call
 * continues the same evolution (for example with a smaller dt) until
 * vp_set_tensors, vp_init_tensors, an update or an optimisation changes the
 * tensors.  On return the lattice's tensors are the evolved PEPS with
 * lambda^(1/2) absorbed into both tensors of every link, and the sampler's
 * boundaries are invalidated as by vp_set_tensors.  change_dev [n_steps]
 * (float64, device, may be NULL) receives App. A's convergence measure per
 * step: the mean over links of ||lambda(t+dt) - lambda(t)|| / ||lambda(t)||.
 * Workspace: the tensors and lambdas of the evolution and the scratch of up
 * to 512 links or diagonals per launch (about 350 KB per link and 2 MB per
 * diagonal at D = 8; at most about 1 GiB), allocated by the first call. */
vp_status vp_simple_update(vp_ctx* ctx, int32_t lat, double dt, int32_t n_steps, double* change_dev);

/* The lambdas of the simple update of the current tensors, lam_dev
 * [n_links][D] float64 (device): horizontal links (y,x)-(y,x+1) row-major,
 * then vertical links (y,x)-(y+1,x) row-major; VP_ERR_ARG when there is none. */
vp_status vp_simple_update_lambdas(vp_ctx* ctx, int32_t lat, double* lam_dev);

/* Integrated autocorrelation time of each chain's measurement series with
 * Sokal's automatic window (Madras & Sokal, J. Stat. Phys. 50, 1988): rho(t)
 * is the normalised autocovariance of the chain, tau(M) = 1/2 + sum_{t=1..M}
 * rho(t), and M is the smallest window with M >= c tau(M).  series_host is
 * [n_chains][len] (host memory); tau_host receives [n_chains].  mean_out is
 * the mean over all samples; stderr_out the standard error of that mean,
 * sqrt(sum_chains var_c 2 tau_c / len) / n_chains.  Host-only, synchronous.
 * Returns VP_ERR_ARG for len < 2 or c <= 0. */
vp_status vp_stats_tau(const double* series_host, int32_t n_chains, int32_t len, double c, double* tau_host,
                       double* mean_out, double* stderr_out);

/* Wait for the context's stream; report device-side error flags. */
vp_status vp_sync(vp_ctx* ctx);

/* Device timing of the sweep phases, for benchmarks and profiling: while
 * enabled, every phase launch is bracketed by a pair of HIP events on the
 * context's stream.  vp_timing_enable clears the accumulated figures;
 * vp_timing_read waits for the stream and writes, per phase, the summed
 * kernel milliseconds and the number of launches (host arrays of VP_NPHASE). */
typedef enum {
  VP_PH_ROW3_ENVS = 0,   /* right 3-line environments of a row (sampling pass) */
  VP_PH_HSWEEP = 1,      /* horizontal Metropolis pass of a row */
  VP_PH_ROW4_ENVS = 2,   /* right 2-row environments (sampling pass) */
  VP_PH_VSWEEP = 3,      /* vertical Metropolis pass between two rows */
  VP_PH_COMPRESS_UP = 4, /* upper boundary U_y */
  VP_PH_COMPRESS_DOWN = 5, /* lower boundary D_y */
  VP_PH_MEASURE3 = 6,    /* log-derivatives and horizontal ratios of a row */
  VP_PH_MEASURE4 = 7,    /* vertical and diagonal ratios of a row pair */
  VP_PH_OTHER = 8,
  VP_NPHASE = 9
} vp_phase;
vp_status vp_timing_enable(vp_ctx* ctx, int32_t enable);
vp_status vp_timing_read(vp_ctx* ctx, double* ms_host, int64_t* launches_host);

#ifdef __cplusplus
}
#endif

#endif /* VMCPEPS_H */
