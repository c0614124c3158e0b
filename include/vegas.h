/*
 * vegas.h -- C ABI of the MI355X (gfx950) VEGAS hot-path library.
 *
 * The library estimates a multi-dimensional integral by VEGAS: iterations of
 * independent events, all events of an iteration combined once, then a serial
 * re-optimisation of the adaptive grid (Campbell, Ellis, Giele, "A
 * Multi-Threaded Version of MCFM", Sec. 2.1; abstract).  Every step of an
 * iteration runs in the library's HIP kernels on the caller's stream.
 *
 * Conventions for every function:
 *   - returns VEGAS_OK (0) or a negative vegas_status; no C++ exception
 *     crosses the ABI; vegas_strerror() gives a message, including the HIP
 *     error text of the last VEGAS_EHIP on that thread;
 *   - a handle is not thread-safe; separate handles are independent;
 *   - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *     pointers are caller-owned device memory on the handle's device, ordered
 *     on the handle's stream.
 *   - results do not depend on the launch configuration (waves per block,
 *     number of blocks): the per-iteration sums are exact integer fixed-point
 *     accumulations, so every launch gives byte-identical numbers (Sec. 2.2:
 *     results independent of the number of threads).
 */
#ifndef VEGAS_H
#define VEGAS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VEGAS_OK = 0,
  VEGAS_EINVAL = -1, /* bad configuration or argument                         */
  VEGAS_ESTATE = -2, /* call order (e.g. refine before any iterate)            */
  VEGAS_ENOMEM = -3, /* workspace too small or device allocation failed        */
  VEGAS_EHIP = -4,   /* HIP runtime error; text kept for vegas_strerror         */
  VEGAS_ETOOBIG = -5 /* request larger than the static scratch of an
                        allocation-free call (VEGAS_SCRATCH_DOUBLES)           */
} vegas_status;

/* integrands (processes) */
typedef enum {
  VEGAS_GAUSS = 0,  /* separable normalised Gaussian on [0,1]^ndim; params (mu, sigma)     */
  VEGAS_GENZ = 1,   /* Genz families 1..6; params (family, a[ndim], w[ndim])                */
  VEGAS_EEMUMU = 2, /* e+e- -> mu+mu- at fixed s, ndim 2                                     */
  VEGAS_DY_Z = 3,   /* q qbar -> photon/Z -> l+l-, hadronic, ndim 3 (m^2 by Breit-Wigner,
                       ln x1, cos theta)                                                    */
  VEGAS_W_PLUS = 4, /* u dbar -> W+ -> e+ nu, hadronic, lepton pT / |eta| cuts, ndim 4      */
  VEGAS_WW_4L = 5,  /* q qbar -> W+W- -> e+ nu mu- nubar, partonic at fixed sqrt(shat),
                       doubly resonant tree amplitudes, ndim 8 = 3*4 - 4 (Sec. 3.2)         */
  VEGAS_WW_HAD = 6  /* the same in pp collisions: the partonic weight at shat = tau S times
                       the parton luminosity, ndim 10 = 3*4 - 4 + 2 momentum fractions
                       (Sec. 3.2: the 3n - 4 integrations plus the two fractions);
                       x8 -> ln tau uniform over the sqrt(shat) window [MLO, MHI] (MHI <= 0:
                       sqrt(S), 0 < MLO < MHI), x9 -> ln x1 = x9 ln tau; both beam orderings
                       as twice the quark-from-beam-1 term (the same integral); binary64
                       only (up to sqrt(S) the diagrams cancel by (shat/M_W^2)^2)          */
} vegas_process;

/* arithmetic of the matrix element */
typedef enum {
  VEGAS_FP64 = 0,    /* everything in binary64                                          */
  VEGAS_FP32_ME = 1  /* WW_4L only: spinors, currents and amplitudes in binary32; mappings,
                        Jacobians, Breit-Wigner, weights, sums and refinement in binary64 */
} vegas_precision;

/* physics parameter vector (processes 2..5), length VEGAS_NPHYS */
enum {
  VEGAS_P_ALPHA = 0,  /* alpha_em                                      */
  VEGAS_P_SW2 = 1,    /* sin^2 theta_W                                 */
  VEGAS_P_MZ = 2, VEGAS_P_GZ = 3, VEGAS_P_MW = 4, VEGAS_P_GW = 5,
  VEGAS_P_SQRTS = 6,  /* hadronic sqrt(S), or sqrt(shat) for EEMUMU/WW_4L */
  VEGAS_P_PDF_A = 7, VEGAS_P_PDF_a = 8, VEGAS_P_PDF_b = 9, /* f(x) = A x^a (1-x)^b */
  VEGAS_P_MLO = 10, VEGAS_P_MHI = 11, /* Breit-Wigner mass window; MHI <= 0: sqrt(S) */
  VEGAS_P_PTMIN = 12, VEGAS_P_ETAMAX = 13, /* charged-lepton cuts (W_PLUS)           */
  VEGAS_P_VUD = 14,
  VEGAS_P_CONV = 15,  /* (hbar c)^2 in pb GeV^2                        */
  VEGAS_NPHYS = 16
};

#define VEGAS_MAX_DIM 16
#define VEGAS_MAX_BINS 255
#define VEGAS_MAX_PARAMS 64
#define VEGAS_MAX_ITER 4096
#define VEGAS_MAX_OBS_BINS 254

typedef struct {
  int32_t process;         /* vegas_process                                          */
  int32_t ndim;            /* GAUSS/GENZ: 1..16; others must equal their dimension   */
  int32_t nbins;           /* bins per dimension, 2..255                              */
  int32_t precision;       /* vegas_precision                                        */
  uint64_t seed;           /* key of the counter-based random numbers                */
  double alpha;            /* grid damping exponent (1.5 typical), >= 0              */
  const double *params;    /* host, copied at init; may be NULL if nparams == 0      */
  int32_t nparams;         /* <= VEGAS_MAX_PARAMS                                     */
  int32_t waves_per_block; /* launch knob: 0 = auto, else 1, 2, 4, 8 or 16            */
  int32_t max_blocks;      /* launch knob: 0 = auto, else cap on blocks per launch    */
} vegas_config;

typedef struct {
  double integral;      /* I_j = S1 / N                                    */
  double variance;      /* var_j = (S2 / N - I_j^2) / (N - 1)              */
  int64_t n_events;     /* N, cut-rejected events included                 */
  int64_t n_nonzero;    /* events with w != 0                              */
  int64_t n_nonfinite;  /* events whose w or w^2 was not finite (dropped)  */
  uint32_t iteration;   /* index j of this iteration (keys the random stream) */
  int32_t fold;         /* how the exact sums were folded: 0 = from the records at
                           this iteration's own scale (first iteration, or the
                           digits do not fit one block's LDS); 1 = inside the
                           event kernel at the scale fixed by the previous
                           iteration (2^16 above its max |w|); 2 = like 1, but
                           this iteration's max |w| left [2^-40, 1) of that scale
                           (or its max w^2 left [2^-40, 1) of the scale of w^2),
                           so the sums were re-folded from the records at the
                           iteration's own scale.  Any fold gives the same
                           integers for every launch configuration. */
} vegas_iter_result;

typedef struct vegas_state *vegas_handle;

/* Device bytes a workspace must hold for cfg and up to max_events per iteration.
 * Errors: VEGAS_EINVAL (bad cfg, max_events < 2 or >= 2^31). */
int vegas_workspace_size(const vegas_config *cfg, int64_t max_events, size_t *bytes);

/* Create a handle: validate cfg, carve device buffers out of `workspace`
 * (device, caller-owned, >= vegas_workspace_size bytes, 256-byte aligned; the
 * library never frees it) or, if workspace is NULL, allocate them itself;
 * set the uniform grid e_k = k / nbins (Sec. 2.1: the grid is then optimised
 * after each iteration).  stream: hipStream_t or NULL for the null stream;
 * the handle is bound to the current device.
 * Errors: VEGAS_EINVAL, VEGAS_ENOMEM, VEGAS_EHIP. */
int vegas_init(const vegas_config *cfg, int64_t max_events, void *workspace, size_t ws_bytes,
               void *stream, vegas_handle *out);

/* One iteration of n_events events at the current grid (Sec. 2.1: the events
 * are generated and evaluated independently, then all events of the iteration
 * are combined).  Event i of iteration j draws its point from the
 * counter-based generator keyed by (seed, j, i) (Sec. 2.2: the same events for
 * any split of the work), maps it through the grid, evaluates the integrand and
 * accumulates w, w^2 and the per-bin histogram of w^2 exactly.  j is the
 * handle's iteration counter, incremented by this call.
 * out (host, nullable): if given, the call waits for the stream and fills it;
 * if NULL the call is asynchronous on the stream.
 * Errors: VEGAS_EINVAL (n_events < 2 or above max_events), VEGAS_ESTATE
 * (more than VEGAS_MAX_ITER iterations), VEGAS_EHIP. */
int vegas_iterate(vegas_handle h, int64_t n_events, vegas_iter_result *out);

/* Re-optimise the grid from the last iteration's histogram (Sec. 2.1: serial
 * grid optimisation between iterations): per dimension, neighbour smoothing,
 * r_k = dbar_k / sum dbar, damping m_k = ((r_k - 1)/ln r_k)^alpha, new edges at
 * equal cumulative m.  The iteration's finalisation normally computes this
 * grid already (into a second buffer) and the call only swaps the buffers;
 * after vegas_set_grid or vegas_set_state it runs as its own kernel.  Either
 * way the result is the same and ordered on the stream.
 * Errors: VEGAS_ESTATE (no iteration since init or since the last refine). */
int vegas_refine(vegas_handle h);

/* A schedule of count iterations (Sec. 3.2: the paper's timing runs are a warm-up
 * stage and a production stage of fixed event counts), iteration j with
 * n_events[j] events and, if refine != 0, vegas_refine after each: the same results,
 * bit for bit, as those calls made one by one.  With small iterations each step is a
 * few short kernels, so the first call records the schedule's launches as a HIP graph
 * on the handle's stream and a later call with the same event counts, from the same
 * host state (iteration index, buffer roles, fold scales, launch settings), replays it
 * with one launch; any other call records anew (one recorded schedule per handle).
 * Stratified or timed handles run the calls one by one.  Asynchronous on the stream.
 * n_events (host, count entries) is read during the call only.
 * Errors: VEGAS_EINVAL (count < 1, an entry < 2 or above max_events), VEGAS_ESTATE
 * (the schedule would exceed VEGAS_MAX_ITER iterations, or a refinement without an
 * iteration), VEGAS_EHIP (also when the recording fails; the handle's state is then
 * unchanged). */
int vegas_run_schedule(vegas_handle h, const int64_t *n_events, int32_t count, int32_t refine);

/* Inverse-variance combination of all iterations so far (Sec. 2.1: several
 * iterations of sets of events): integral, its error and chi^2 per degree of
 * freedom.  If an iteration has zero variance the plain mean of such
 * iterations is returned with error 0.  Waits for the stream; host outputs.
 * Errors: VEGAS_ESTATE (no iteration yet). */
int vegas_result(vegas_handle h, double *integral, double *error, double *chi2_dof,
                 int32_t *n_iter);

/* The same combination over iterations first .. (last) only.  The timing runs
 * of Sec. 3.2 use a two-stage schedule (a few small iterations, then larger
 * ones); whether the first stage enters the result is not stated, and this
 * call lets a caller drop it (first = number of warm-up iterations; first = 0
 * is vegas_result).  n_iter receives the number of iterations combined.
 * Errors: VEGAS_ESTATE (no iteration yet), VEGAS_EINVAL (first < 0 or first
 * not below the number of iterations done). */
int vegas_result_from(vegas_handle h, int32_t first, double *integral, double *error,
                      double *chi2_dof, int32_t *n_iter);

/* Stratified sampling on top of the importance grid (Lepage's stratified +
 * importance mode; the paper cites VEGAS (Sec. 2.1) but does not say which mode
 * MCFM runs): strata_per_axis = m cuts the unit cube of the grid's inputs into
 * H = m^ndim equal hypercubes (0 turns it off, the default).  An iteration asked
 * for n events then uses npc = floor(n / H) >= 2 events in every hypercube, so
 * H npc events in all (reported in n_events; refused with VEGAS_EINVAL if
 * npc < 2); event i lies in hypercube floor(i / npc), whose coordinates are the
 * base-m digits of its index (dimension 0 the least significant), and its
 * uniforms r are placed inside it, u = (c + r) / m, before the grid map.  The
 * estimate stays the mean of the weights (equal counts per hypercube); its
 * variance becomes sum_h (1/H)^2 sigma_h^2 / npc with sigma_h^2 the sample
 * variance of the weights in hypercube h (exact, launch-independent sums).  The
 * grid histogram is unchanged.  Not with the learned proposal
 * (vegas_iterate_flow refuses while it is set).  Errors: VEGAS_EINVAL (m < 0,
 * or m^ndim above 2^31 - 1). */
int vegas_set_strata(vegas_handle h, int32_t strata_per_axis);

/* Adaptive allocation over the hypercubes (a reading of Lepage's VEGAS+ adaptive
 * stratification): beta > 0 gives each hypercube of an iteration of n events
 * n_h = 2 + floor((n - 2H) p_h / sum p) events, p_h = sigma_h^beta with sigma_h the
 * standard deviation of the weight in h in the last stratified iteration (beta = 1:
 * Neyman's allocation n_h ~ sigma_h), and the remaining R events one each to
 * hypercubes 0 .. R - 1, so all n events are used (n >= 2H required); equal counts
 * before any stratified iteration, after vegas_set_strata / vegas_set_state, if
 * every p_h is 0, or if rounding made the floors exceed n - 2H.  Each weight is then
 * scaled by N / (H n_h), the volume its event stands for, so the estimate stays the
 * mean and var_j = sum_h n_h sigma_h^2(scaled) / N^2.  The sums are exact as for
 * equal counts; the allocation's own sum of p_h is a fixed-order binary64 sum.
 * beta = 0 (the default) is the equal-count mode of vegas_set_strata.  The
 * allocation scratch (about 16 bytes per hypercube and 4 per event) is allocated by
 * the library on first use.  Errors: VEGAS_EINVAL (beta < 0 or not finite). */
int vegas_set_strata_beta(vegas_handle h, double beta);

/* Events per hypercube of the last stratified iteration, host int32 [m^ndim].
 * Waits for the stream.  Errors: VEGAS_ESTATE (no stratified iteration since
 * vegas_set_strata / vegas_set_state). */
int vegas_get_strata_counts(vegas_handle h, int32_t *counts);

/* Histogram of the process's observable, filled by the same events and weights
 * as the integral (Sec. 2.1: the integrator returns cross sections and
 * distributions of kinematic variables; Sec. 3.2 shows such distributions, the
 * di-jet mass, from production runs, while its timing runs fill no histograms).
 * The observable: x_0 (GAUSS, GENZ), cos(theta) of the mu- (EEMUMU), the
 * lepton-pair mass (DY_Z), the e+ transverse momentum, taken before the cuts
 * (W_PLUS), the e+ nu mass (WW_4L).  nbins (0..VEGAS_MAX_OBS_BINS; 0 turns it
 * off) uniform bins on [lo, hi) (finite, lo < hi), plus an underflow bin
 * (index 0, below lo) and an overflow bin (index nbins + 1, at or above hi);
 * an event falls in bin floor((o - lo) * (nbins / (hi - lo))) + 1, the factor
 * rounded once.  Each bin is the iteration's sum of w over its events divided
 * by N, with error sqrt((S2_b / N - H_b^2) / (N - 1)); its sums are exact and
 * launch-independent like the total's.  Iterations numbered >= first_iteration
 * (the iteration counter) are combined bin by bin with the integral's weights
 * 1 / var_j (the plain mean if an iteration has zero variance), so the bins of
 * the combination add up to the combined integral over the same iterations.
 * Clears the combination; takes effect from the next iteration.  Records one
 * byte per event and six digit columns per bin.
 * Errors: VEGAS_EINVAL. */
int vegas_set_observable(vegas_handle h, int32_t nbins, double lo, double hi,
                         int32_t first_iteration);

/* Last iteration's histogram and its errors, and the combination and its errors:
 * host arrays of nbins + 2 (underflow first, overflow last), each nullable.
 * Waits for the stream.  Errors: VEGAS_ESTATE (no observable set, or no
 * iteration since it was set or since vegas_set_state). */
int vegas_get_observable(vegas_handle h, double *last, double *last_err, double *comb,
                         double *comb_err);

/* Grid edges, host array [ndim][nbins+1] (waits for the stream). */
int vegas_get_grid(vegas_handle h, double *edges);
/* Replace the grid (host [ndim][nbins+1]; e_0 = 0, e_n = 1, non-decreasing).
 * Errors: VEGAS_EINVAL. */
int vegas_set_grid(vegas_handle h, const double *edges);

/* Last iteration's per-bin histogram d [ndim][nbins] (sum of w^2 over the
 * events in each bin) and sums {S1, S2}; host arrays.  Errors: VEGAS_ESTATE. */
int vegas_get_hist(vegas_handle h, double *d, double *sums);

/* Weights of events [first, first+n) of the last iteration, host w[n], and
 * their bin indices, host bins[n][ndim] (nullable).  Errors: VEGAS_EINVAL,
 * VEGAS_ESTATE. */
int vegas_get_weights(vegas_handle h, int64_t first, int64_t n, double *w, uint8_t *bins);

/* Checkpoint: grid, iteration counter and the per-iteration estimates.
 * vegas_get_state with buf == NULL sets *bytes to the size needed.  A restored
 * handle continues bit-identically, because events are keyed by (seed, j, i).
 * The observable histogram is not part of it: vegas_set_state keeps the
 * handle's binning and clears the combination.
 * Errors: VEGAS_EINVAL (size or configuration mismatch). */
int vegas_get_state(vegas_handle h, void *buf, size_t *bytes);
int vegas_set_state(vegas_handle h, const void *buf, size_t bytes);

/* Change the launch configuration (must not change any result). */
int vegas_set_launch(vegas_handle h, int32_t waves_per_block, int32_t max_blocks);

/* Per-stage kernel timing (off by default).  stages is a mask over the four
 * stages {events (k_event, with the fused fold) = VEGAS_TIME_EVENTS, fold (the
 * column sums of the per-block partial rows, and the first iteration's fold
 * from the records) = VEGAS_TIME_FOLD, finalisation (estimate, next scales,
 * speculative refinement) = VEGAS_TIME_FINAL, refinement (only when it runs as
 * its own kernel) = VEGAS_TIME_REFINE}; 0 turns timing off.  Every kernel of a
 * selected stage is launched with a start and a stop HIP event bound to its
 * own dispatch (hipExtLaunchKernel), so timing adds no work between kernels; it
 * does add host time per launch, which a long kernel (the event kernel) hides
 * and a short one may not.  vegas_stage_times waits for the stream and returns
 * the summed kernel milliseconds ms[4] and kernel counts launches[4] per stage
 * (host arrays, either nullable) since the last reset; reset != 0 clears them.
 * vegas_grad's kernels count in the same stages: its event kernel as events,
 * its tree reduction as fold, its output kernel as finalisation.
 * Errors: VEGAS_EINVAL (stages outside 0 .. VEGAS_TIME_ALL). */
enum {
  VEGAS_TIME_EVENTS = 1, VEGAS_TIME_FOLD = 2, VEGAS_TIME_FINAL = 4, VEGAS_TIME_REFINE = 8,
  VEGAS_TIME_ALL = 15
};
int vegas_set_timing(vegas_handle h, int32_t stages);

/* Launch shape of the last iteration: info[0] event-kernel blocks, info[1]
 * threads per block, info[2] rows of per-block partials folded, info[3] int64
 * columns per row (7 + 4 ndim nbins: three digits of S1, four of S2 and of each
 * grid-histogram bin; plus seven per observable bin, under- and overflow
 * included, when an observable histogram is set); host array of 4.
 * Errors: VEGAS_EINVAL, VEGAS_ESTATE (no iteration yet). */
int vegas_last_launch(vegas_handle h, int64_t *info);
int vegas_stage_times(vegas_handle h, double *ms, int64_t *launches, int32_t reset);

/* Adjoint of the Drell-Yan estimator (process VEGAS_DY_Z only).  For B parameter
 * points theta_b = (M_Z, Gamma_Z, sin^2 theta_W, PDF a, PDF b) (device, [B][5],
 * 1 <= B <= 64) computes sigma_b = (1/N) sum_i w_i(theta_b) and its gradient
 * dsigma_b/dtheta (device outputs sigma[B], dsigma[B][5]) over events
 * i < n_events of iteration index `iteration` at the handle's current grid:
 * common random numbers for all points, the proposal (grid, Breit-Wigner and
 * tau mappings) held at the handle's nominal parameters, a hand-written reverse
 * sweep through |M|^2 and the PDFs per (event, point).  Results do not depend
 * on the launch configuration.  Asynchronous on the stream; scratch of
 * 8 * 6 * B * (ceil(n/64) + ceil(n/16384)) bytes is allocated by the library on
 * first use and kept until vegas_destroy.  (Paper Sec. 2.1 fixes the estimator;
 * the derivative is this library's extension.)
 * Errors: VEGAS_EINVAL (other process, B or n out of range, NULL), VEGAS_ENOMEM. */
int vegas_grad(vegas_handle h, const double *params_dev, int32_t B, int64_t n_events, uint32_t iteration,
               double *sigma_dev, double *dsigma_dev);

/* vegas_grad without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid it.
 * Same arguments, kernels, results (bit for bit) and errors as vegas_grad, but
 * the per-tile partials and the tree's first level live in a static device
 * array of VEGAS_SCRATCH_DOUBLES binary64 values (16 MiB) that the library
 * holds on each GPU it runs on until the process ends; a call needs
 * (T + ceil(T / 256)) * 6 * B of them, T = ceil(n_events / 64) (at B = 64 up
 * to about 3.4e5 events, at B = 8 about 2.7e6).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * handles) race and give wrong results; calls ordered on one stream do not.
 * Errors: as vegas_grad; VEGAS_ETOOBIG above the scratch size; VEGAS_EHIP if
 * the array's device address could not be taken when the handle was made. */
#define VEGAS_SCRATCH_DOUBLES (1u << 21)
int vegas_grad_noalloc(vegas_handle h, const double *params_dev, int32_t B, int64_t n_events,
                       uint32_t iteration, double *sigma_dev, double *dsigma_dev);

/* Release the handle (and the buffers the library allocated itself). */
int vegas_destroy(vegas_handle h);

/* ------------------------------------------------------------------------
 * Learned proposal (this library's extension; the paper's proposal is the
 * VEGAS grid of Sec. 2.1).  A normalising flow q on the unit hypercube
 * [0,1]^8 that the grid map is applied to: six coupling layers, each mapping
 * four coordinates by monotone rational-quadratic splines (16 bins) whose
 * parameters an MLP 4 -> 128 -> 128 -> 188 (ReLU) computes from the other four
 * (Durkan et al., Neural Spline Flows, 2019).  The MLP runs in bfloat16 with
 * binary32 accumulation on the matrix cores; splines, log-densities and the
 * FP32 master weights are binary32.  A flow iteration draws z uniform from
 * the same counter-based stream as a VEGAS iteration, y = F^{-1}(z), x = the
 * grid map of y, and weights w = f(x) J(y) / q(y): an unbiased estimate of the
 * same integral for any flow parameters.
 *
 * Flat parameter vector (binary32, 248424 values), per layer l = 0..5 in
 * order: W1 [4][128], b1 [128], W2 [128][128], b2 [128], W3 [128][188],
 * b3 [188] (input-major).  Layer l transforms the coordinates
 * {4567},{0123},{1357},{0246},{2367},{0145} (l = 0..5) and is conditioned on
 * the other four in increasing order; the 188 outputs are, per transformed
 * coordinate in increasing order, 16 width logits, 16 height logits and 15
 * interior-derivative pre-activations.
 * ---------------------------------------------------------------------- */
typedef struct vegas_flow_state *vegas_flow;

#define VEGAS_FLOW_NPARAMS 248424

/* Create a flow: He-uniform hidden layers from the counter-based generator
 * keyed by seed, zero output layer (the identity map, q = 1).  max_batch
 * (1 .. 2^22) bounds the batch of the density / training calls; max_sample
 * (0 .. 2^31-1) the events of a flow iteration.  The library allocates
 * about 3.4 KB per batch event plus 36 B per sample event plus 5 MB of
 * device memory, freed by vegas_flow_destroy.  stream: hipStream_t or NULL.
 * Errors: VEGAS_EINVAL, VEGAS_ENOMEM, VEGAS_EHIP. */
int vegas_flow_create(int32_t max_batch, int64_t max_sample, uint64_t seed, void *stream, vegas_flow *out);
int vegas_flow_destroy(vegas_flow f);

/* Copy the FP32 master parameters out (device dst [VEGAS_FLOW_NPARAMS]) or in
 * (device src; refreshes the bfloat16 copies and resets the optimiser moments
 * and step count).  Asynchronous.  Errors: VEGAS_EINVAL, VEGAS_EHIP. */
int vegas_flow_get_params(vegas_flow f, float *dst_dev);
int vegas_flow_set_params(vegas_flow f, const float *src_dev);

/* log q(y) for B points (device y [B][8] in [0,1], device logq [B]),
 * 1 <= B <= max_batch.  Asynchronous.  Errors: VEGAS_EINVAL, VEGAS_EHIP. */
int vegas_flow_density(vegas_flow f, const float *y_dev, int64_t B, float *logq_dev);

/* Loss L = -sum_i w_i log q(y_i) / sum_i w_i over B weighted points (device y
 * [B][8], device w [B], w >= 0 with a positive sum) and its gradient with
 * respect to the parameters, written to device grad [VEGAS_FLOW_NPARAMS]
 * (nullable).  loss (host, nullable): if given, the call waits for the stream.
 * Errors: VEGAS_EINVAL, VEGAS_EHIP. */
int vegas_flow_loss_grad(vegas_flow f, const float *y_dev, const double *w_dev, int64_t B, float *grad_dev,
                         double *loss_host);

/* One Adam step (beta = 0.9, 0.999, eps = 1e-8, learning rate lr) on a batch
 * of `batch` points of a data set of n_data (1 .. 2^31-1) weighted points
 * (device y [n_data][8], w [n_data]).  Step s takes positions [(s mod m) batch, ...) of
 * epoch floor(s / m), m = ceil(n_data / batch), through a per-epoch
 * permutation i -> (a i + c) mod n_data (wrapping at the end of the data).
 * loss (host, nullable) as for vegas_flow_loss_grad.
 * Errors: VEGAS_EINVAL, VEGAS_EHIP. */
int vegas_flow_train_step(vegas_flow f, const float *y_dev, const double *w_dev, int64_t n_data, int32_t batch,
                          uint64_t step, float lr, double *loss_host);

/* Sampling direction: y = F^{-1}(z) and log q(y) for n points (device z, y
 * [n][8], y may equal z; device logq [n]).  Asynchronous.
 * Errors: VEGAS_EINVAL, VEGAS_EHIP. */
int vegas_flow_sample(vegas_flow f, const float *z_dev, int64_t n, float *y_dev, float *logq_dev);

/* Training data from the last iteration of h (a VEGAS iteration, not a flow
 * one): events [first, first+n) as device y [n][8] (binary32 rounding of the
 * event's uniform point, before the grid map) and device w [n] (its weight).
 * Requires ndim = 8.  Asynchronous.
 * Errors: VEGAS_EINVAL (range, ndim), VEGAS_ESTATE (no VEGAS iteration yet,
 * or the last iteration used the flow). */
int vegas_export(vegas_handle h, int64_t first, int64_t n, float *y_dev, double *w_dev);

/* One iteration with the flow as proposal: z_i from the stream keyed by
 * (seed, j, i) as in vegas_iterate, y_i = F^{-1}(z_i), then the same grid map,
 * integrand, exact accumulation and combination as vegas_iterate, with
 * w_i = f(x_i) J(y_i) exp(-log q(y_i)).  The grid is frozen: vegas_refine after
 * a flow iteration returns VEGAS_ESTATE.  Requires ndim = 8 and
 * n_events <= the flow's max_sample.  The flow's work is ordered on the
 * handle's stream after the flow's own stream.  out as for vegas_iterate.
 * Errors: as vegas_iterate. */
int vegas_iterate_flow(vegas_handle h, vegas_flow f, int64_t n_events, vegas_iter_result *out);

/* Message for a status code. */
const char *vegas_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
