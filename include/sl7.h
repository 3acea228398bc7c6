/*
 * sl7.h -- C ABI of the MI355X (gfx950) Seven-League (7L) library.
 *
 * The library runs the online stage of the 7L scheme (arXiv 2302.05170,
 * Algorithm I, steps 2-8): every Monte Carlo path takes M large steps; at each
 * step the collocation network H maps (Y_i, dt, theta) to m collocation
 * points y_j (eq. 6.3/6.4), a fresh standard normal X is drawn and
 * Y_{i+1} = g_m(X), the barycentric Lagrange interpolant through (x_j, y_j)
 * with x_j the Gauss-Hermite points of N(0,1) (Methodology and
 * Parallelization sections).  Beside it: the offline stage that makes labels
 * and trains H (Algorithm I, step 1), a reverse-mode adjoint for pathwise
 * sensitivities, and a batched launch over many uneven instances.
 *
 * Conventions shared by every entry point:
 *   - Every call returns an int status: SL7_OK (0) or a negative SL7_E* code.
 *     sl7_last_error() then gives a message naming the offending argument.
 *     The message is thread-local and valid until the next call on the same
 *     thread.  No C++ exception crosses this boundary.  On error the contents
 *     of output buffers are unspecified.
 *   - "device" pointers are HIP device allocations owned by the caller, on the
 *     current HIP device; "host" pointers are ordinary host memory owned by
 *     the caller.  The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it; calls that return results into host memory
 *     synchronise that stream before returning, as documented per call.
 *     Calls on one device share its internal buffers; the library orders
 *     each call's work after the previous call's with an event, so calls
 *     that do not synchronise may be issued from several threads on several
 *     streams (their device work then runs one call after another).
 *   - A network handle may be read by several calls at once (simulation,
 *     evaluation, adjoint).  Calls that change or free it (sl7_mlp_set_params,
 *     sl7_train, sl7_mlp_free) must not overlap any other call that uses the
 *     same handle; work already enqueued with it completes before its device
 *     copies are released.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit
 *     seed, counter (step/4, path low word, path high word, tag) with
 *     tag = domain << 24 | instance, domain 0 for simulation and 1 for
 *     labels; Box-Muller turns each call's four words into four normals for
 *     four consecutive steps.  Paths use global indices, so results do not
 *     depend on how paths are tiled over the GPU.
 *   - Model parameter vectors theta[]: GBM dY = mu Y dt + sigma Y dW with
 *     theta = (sigma, mu); OU (eq. 6.5) with theta = (ybar, sigma, lambda);
 *     CIR dY = kappa (ybar - Y) dt + gamma sqrt(Y) dW with
 *     theta = (kappa, ybar, gamma).  The network's inputs are
 *     (Y, dt, theta[0], ..., theta[n-1]) in that order.
 */
#ifndef SL7_H
#define SL7_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define SL7_OK 0
#define SL7_EINVAL (-1)       /* an argument is out of range or inconsistent */
#define SL7_EUNSUPPORTED (-2) /* valid request the library does not implement */
#define SL7_EHIP (-3)         /* a HIP runtime call failed */
#define SL7_ENOMEM (-4)       /* device or host allocation failed */
#define SL7_ENUMERIC (-5)     /* non-finite weights or results */
#define SL7_EIO (-6)          /* weight file could not be read or written */

/* Models (eq. 6.1 specialised). */
#define SL7_GBM 0
#define SL7_OU 1
#define SL7_CIR 2

/* Arithmetic of the network GEMMs.  F64: everything in double.  F32: GEMMs
 * on FP32 MFMA.  BF16 / F16: hidden-layer and head GEMM operands rounded
 * (RNE) once to bfloat16 / half, one MFMA pass with FP32 accumulation.
 * BF16X3 / F16X3: the same MFMA instructions on split operands
 * x = hi + lo (hi = x rounded to 16 bits -- to nearest, except BF16
 * activations, which are truncated -- and lo = rn16(x - hi)) for weights and
 * activations, three passes hi*hi + hi*lo + lo*hi accumulated in FP32
 * (close to FP32 accuracy; the one-pass forms carry a rounding bias per
 * step).  In every mode the first layer, the interpolation and the state
 * update stay FP32 and the path mean is reduced in FP64.
 *
 * PWL32 / PWL64 (ReLU networks only): no GEMMs in the loop.  For a fixed
 * instance the network's only varying input is Y, and a ReLU network is then
 * an exactly piecewise-linear function of Y (each unit is affine on either
 * side of one breakpoint, layer after layer).  The library compiles that
 * function per instance on the host in FP64 (at most 65536 pieces, else
 * SL7_EUNSUPPORTED) and each path evaluates y_j = c_j + a_j (Y - o) on its
 * piece, found through a uniform grid over the breakpoints; lane arithmetic
 * (piece search, y_j, interpolation, update) in FP32 or FP64.  Mathematically
 * identical to evaluating the network, to rounding. */
/* Precision codes are plain int arguments (named `prec`): an int has the
 * same size and passing convention under every C and C++ compiler, which a
 * C enum type does not guarantee across a shared-library boundary. */
#define SL7_F64 0
#define SL7_F32 1
#define SL7_BF16 2
#define SL7_F16 3
#define SL7_BF16X3 4
#define SL7_F16X3 5
#define SL7_PWL32 6
#define SL7_PWL64 7

/* Hidden activations. */
#define SL7_RELU 0
#define SL7_SOFTPLUS 1

/* Largest sizes the kernels accept. */
#define SL7_MAX_M 8       /* collocation points */
#define SL7_MAX_DIN 8     /* network inputs */
#define SL7_WIDTH 64      /* hidden width the kernels are built for */
#define SL7_DEPTH 4       /* hidden layers the kernels are built for */

typedef struct sl7_mlp sl7_mlp; /* opaque network handle */

/* Network description: d_in inputs -> depth hidden layers of `width` units
 * -> m outputs.  h0 = in_scale * input + in_shift (elementwise), so the
 * inputs' training ranges can be mapped to [-1, 1]; dom_lo/dom_hi record the
 * training domain (used to count out-of-domain network calls). */
typedef struct {
  int32_t d_in, width, depth, m, act, model;
  double in_scale[SL7_MAX_DIN], in_shift[SL7_MAX_DIN];
  double dom_lo[SL7_MAX_DIN], dom_hi[SL7_MAX_DIN];
} sl7_mlp_desc;

/* One simulation instance (Algorithm I, online stage).  dt = T / M,
 * t_i = i T / M.  Paths path_offset .. path_offset + N - 1 (global indices,
 * used as the Philox counter; path_offset >= 0, path_offset + N <= 2^63 - 1,
 * 1 <= N <= 2^40, else SL7_EINVAL).  instance becomes the low 24 bits of the
 * tag. */
typedef struct {
  int32_t model, m, M, reserved0;
  int64_t N;
  double theta[4];
  double Y0, T, K; /* K: strike of the second payoff max(Y_T - K, 0) */
  int64_t path_offset;
  uint32_t instance, reserved1;
} sl7_problem;

/* Results for two payoffs: index 0 is Y_T, index 1 is max(Y_T - K, 0).
 * var uses N - 1; se = sqrt(var / N).  n_clamped counts CIR steps whose
 * interpolated value was negative and was set to 0; n_out_of_domain counts
 * network evaluations whose Y input lay outside the training domain. */
typedef struct {
  double mean[2], var[2], se[2];
  int64_t n, n_clamped, n_out_of_domain, reserved;
} sl7_stats;

/* Launch plan of the fused kernel.  A plan changes speed, never results. */
typedef struct {
  int32_t waves_per_block; /* 1, 2 or 4 wave64s per workgroup; also 12 in the split
                              modes SL7_BF16X3 / SL7_F16X3 (all weights in LDS, three
                              waves per SIMD; the default there from 64 blocks of
                              64 paths per compute unit) */
  int32_t blocks_per_cu;   /* persistent grid = blocks_per_cu x compute units */
  int32_t grab;            /* 64-path blocks taken per work-queue grab */
  int32_t reserved;
} sl7_plan;

/* --- errors ---------------------------------------------------------- */
const char* sl7_last_error(void);
const char* sl7_version(void);

/* --- collocation nodes (Methodology section: x_j from N(0,1)) ---------- */
/* Probabilists' Gauss-Hermite nodes (roots of He_m), ascending and
 * symmetric, and weights w_j summing to 1.  m in [1, 16].  x, w: host,
 * m doubles each. */
int sl7_gh_nodes(int m, double* x, double* w);

/* --- the network H (eq. 6.3/6.4) -------------------------------------- */
/* Number of FP32 parameters of a description: per layer W (out x in,
 * row-major) then b, layers in order. */
int64_t sl7_mlp_n_params(const sl7_mlp_desc* d);
/* Creates a handle from a description and a host parameter vector (copied).
 * EINVAL on bad dimensions, ENUMERIC on non-finite parameters. */
int sl7_mlp_create(const sl7_mlp_desc* d, const float* params, sl7_mlp** H);
/* Reads / writes the little-endian weight file ("SL7W" version 1: u32
 * version, d_in, width, depth, m, act, model; f64 in_scale, in_shift,
 * dom_lo, dom_hi [d_in each]; per layer f32 W then b; u32 length and JSON
 * metadata).  EIO on unreadable files, EINVAL on malformed ones. */
int sl7_mlp_load(const char* path, sl7_mlp** H);
int sl7_mlp_save(const sl7_mlp* H, const char* path);
/* Copies the description / current parameters out (host memory). */
int sl7_mlp_get_desc(const sl7_mlp* H, sl7_mlp_desc* d);
int sl7_mlp_get_params(const sl7_mlp* H, float* params);
/* Replaces the parameters (host vector, copied; device copies refreshed). */
int sl7_mlp_set_params(sl7_mlp* H, const float* params);
void sl7_mlp_free(sl7_mlp* H);

/* Batched forward pass of H (Algorithm I step 3, eq. 6.4): in [B x d_in]
 * raw inputs, row-major FP32, device; out [B x m] FP32, device.  prec as
 * above.  Asynchronous on `stream`. */
int sl7_eval_H(const sl7_mlp* H, int prec, const float* in_dev, int64_t B,
               float* out_dev, void* stream);

/* --- the online stage (Algorithm I, steps 2-8) ------------------------- */
/* Simulates pr->N paths of pr->M steps.  H == NULL selects the analytic
 * collocation map of the model (GBM: y_j = Y exp((mu - sigma^2/2) dt +
 * sigma sqrt(dt) x_j); OU: eq. 6.6 over one step); otherwise H (whose m
 * and d_in = 2 + n_theta must match).  prec: SL7_F64 for either map; F32
 * for either map; BF16, F16, BF16X3 and F16X3 for the network only; PWL32
 * and PWL64 for ReLU networks only (SL7_EUNSUPPORTED otherwise).
 * YT_dev: NULL, or device buffer of N values (double in F64 and PWL64 modes,
 * float otherwise) that receives Y_T per path.  stats_host: NULL or host struct;
 * when non-NULL the call synchronises `stream` before returning.
 * plan: NULL for the default/tuned plan. */
int sl7_simulate(const sl7_problem* pr, const sl7_mlp* H, int prec,
                 uint64_t seed, void* YT_dev, sl7_stats* stats_host,
                 const sl7_plan* plan, void* stream);

/* The 7L-CDC variant (Numerical Results, after Table 6.1; Parallelization
 * section): the collocation map (H, or the analytic map when H == NULL) is
 * evaluated only at m marginal collocation points per step,
 * s_k = map(Y0 over [0, t_i])_k, and at the conditional points there,
 * y_kj = map(s_k over dt)_j; each path takes y_j(Y_i) by barycentric
 * interpolation in Y over the s_k (a global interpolation instead of a
 * per-path network call) and then Y_{i+1} = g_m(X) as in 7L.  Step 0
 * uses map(Y0 over dt).  The tables are built on the GPU in FP64 (m + 1
 * map evaluations per step, one workgroup per step); the per-path work runs
 * one path per lane in prec SL7_F64 or SL7_F32 (others: SL7_EUNSUPPORTED).
 * Problem, seed (same normals as sl7_simulate), YT_dev and stats_host as in
 * sl7_simulate; stats_host->n_out_of_domain counts the table's network
 * inputs outside the training domain.  Synchronises `stream` (the table
 * checks): SL7_ENUMERIC when two marginal points of a step coincide or a
 * table entry is not finite. */
int sl7_simulate_cdc(const sl7_problem* pr, const sl7_mlp* H, int prec, uint64_t seed,
                     void* YT_dev, sl7_stats* stats_host, void* stream);

/* sl7_simulate for callers that cannot allocate device memory: code under
 * stream (graph) capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same problem, network, prec (every mode but PWL32 / PWL64,
 * which return SL7_EUNSUPPORTED), seed, YT_dev and plan as sl7_simulate,
 * same kernels and bit-identical results.  stats_dev: NULL, or a device
 * sl7_stats that receives the statistics; nothing is copied to the host and
 * the call never synchronises `stream`.  Scratch: one fixed 16.06 MiB array
 * per device inside this library (held until the process ends), so
 * pr->N <= 2^24 (SL7_EINVAL beyond).  H's device copy for prec must already
 * exist on the current device (any earlier sl7_simulate or sl7_eval_H call
 * with H and prec makes it; SL7_EINVAL otherwise).  The call allocates no
 * device or pinned memory.  All calls on one device share the one array:
 * calls whose device work overlaps (other streams, other threads) race;
 * order them on one stream. */
int sl7_simulate_noalloc(const sl7_problem* pr, const sl7_mlp* H, int prec,
                         uint64_t seed, void* YT_dev, sl7_stats* stats_dev,
                         const sl7_plan* plan, void* stream);

/* The piecewise-linear form of a ReLU network H for one instance pr (the
 * SL7_PWL32 / SL7_PWL64 modes above), computed on the host in FP64.
 * *n_pieces receives the piece count P.  With brk/anchor/slope/value all
 * non-NULL (host arrays of P-1, P, P*m and P*m doubles) they receive the
 * breakpoints (ascending; piece p covers [brk[p-1], brk[p])), the anchors
 * o_p and, for output j, y_j = value[p*m+j] + slope[p*m+j] (Y - o_p).  Pass
 * them all NULL to query P.  max_pieces in [1, 65536] caps P
 * (EUNSUPPORTED beyond it; EINVAL for max_pieces outside that range).
 * No device work. */
int sl7_pwl_compile(const sl7_mlp* H, const sl7_problem* pr, int max_pieces, int* n_pieces,
                    double* brk, double* anchor, double* slope, double* value);

/* Many instances of uneven size in one persistent launch (network map,
 * every prec but F64; all instances share m).  Work is 64-path blocks
 * ordered longest-M first and handed out by an atomic work counter; per-instance statistics go to
 * stats_host[n] (synchronises the stream).  With use_graph != 0 the launch
 * sequence is captured once into a hipGraph, with buffers of its own, and
 * replayed by later calls whose problems, plan, seed, prec, device and
 * network weights are all the same (a change of H's parameters makes a new
 * capture); at most 8 captures are kept. */
int sl7_simulate_batched(const sl7_problem* prs, int n, const sl7_mlp* H,
                         int prec, uint64_t seed, sl7_stats* stats_host,
                         const sl7_plan* plan, int use_graph, void* stream);

/* --- reverse-mode sensitivities ---------------------------------------- */
/* Pathwise sensitivities of E[f(Y_T)] (f = Y_T for payoff 0, max(Y_T-K, 0)
 * for payoff 1) to Y0 and theta, by a reverse (adjoint) sweep through all M
 * steps of every path: the forward pass stores Y every ckpt_every steps,
 * the reverse pass recomputes the states in between from the same Philox
 * counters.  grad[0] = dE/dY0, grad[1 + k] = dE/dtheta_k; *_se are the
 * Monte Carlo standard errors of the pathwise estimators.  f'(K) = 0 for
 * the call; ReLU'(0) = 0; a clamped CIR step passes no gradient. */
typedef struct {
  double value, value_se;
  double grad[5], grad_se[5];
  int32_t n_grad, reserved;
} sl7_greeks;

/* Workspace size (bytes) for sl7_adjoint: checkpoints
 * ceil(M / ckpt_every) x N states, the per-step evaluation state of the
 * steps kept at once (in F32 and BF16X3 ckpt_every x N x 128 bytes: two
 * segments of 16-byte records for each of a path's four lanes; in F64
 * ckpt_every x N x 32 bytes: one segment's ReLU masks; in the PWL modes 4
 * bytes of piece index per path-step; the analytic map needs none but the
 * size does not depend on H) plus block sums.  0 for bad arguments. */
size_t sl7_adjoint_ws_bytes(const sl7_problem* pr, int prec, int ckpt_every);

/* H == NULL: analytic map (GBM, OU).  prec: SL7_F64, SL7_F32 or SL7_BF16X3
 * (the accumulation of the theta-gradients is FP64 in all), with the analytic
 * map, a ReLU network or a Softplus network (whose reverse pass recomputes
 * each hidden layer's pre-activation from Y_i for the logistic derivative).
 * In SL7_F32 a network's sweep runs on MFMA with FP32 operands, forward and
 * transposed products over 16-path tiles; SL7_BF16X3 (a network only) runs
 * the same sweep with three-pass split BF16 products (hi*hi + hi*lo + lo*hi
 * of weights and of activations or cotangents, FP32 accumulation).  In both
 * the forward half takes the arithmetic of sl7_simulate's kernel of that
 * precision, so f per path equals the payoff of its Y_T.  SL7_F64 runs one
 * path per lane on the FP64 vector units.  For a ReLU network also
 * SL7_PWL64 / SL7_PWL32, which back-propagate through the network's
 * piecewise-linear form: per piece the slope in Y and dy_j/dtheta_k (the
 * piece's activation pattern held fixed, as back-propagation holds its ReLU
 * masks) are compiled on the host in FP64 with the pieces.  ws_dev: caller's
 * device workspace of at least sl7_adjoint_ws_bytes.  per_path_dev: NULL or
 * device [N x (2 + n_theta)] doubles receiving (f, df/dY0, df/dtheta...)
 * per path.  ckpt_every in [1, 32].  Synchronises `stream`. */
int sl7_adjoint(const sl7_problem* pr, const sl7_mlp* H, int prec, uint64_t seed,
                int payoff, int ckpt_every, sl7_greeks* out_host, double* per_path_dev,
                void* ws_dev, size_t ws_bytes, void* stream);

/* --- offline stage (Algorithm I, step 1) ------------------------------- */
/* Training labels: for each of the n rows of feats_dev ([n x d_in] FP32,
 * device; row = (Y, dt, theta...), d_in = 2 + n_theta(model)), n_paths
 * Euler-Maruyama paths (eq. 6.2, FP64) of `substeps` steps of dt/substeps
 * from Y; labels_dev[r*m + j] (FP32, device) is the empirical quantile of
 * the endpoints at Phi(x_j), linear between order statistics at
 * h = (n_paths - 1) Phi(x_j).  Philox domain 1, counter word 2 =
 * label0 + r.  n_paths in [2, 16384].  Asynchronous on `stream`. */
int sl7_labels(int model, int m, const float* feats_dev, int64_t n, int n_paths,
               int substeps, uint64_t seed, int64_t label0, float* labels_dev,
               void* stream);

/* Adam on the mean squared error over batch x m (the paper's offline
 * training: Glorot start is the caller's parameter vector, batch and
 * learning rate from spec). */
typedef struct {
  int32_t epochs, batch;
  double lr, beta1, beta2, eps;
} sl7_train_spec;

/* Trains H in place (FP32 forward/backward kernels, deterministic gradient
 * sums).  H: 4 hidden layers of at most 64 units, ReLU or Softplus
 * (EUNSUPPORTED otherwise).  X_dev [n x d_in] raw inputs, Y_dev [n x m]
 * labels (device, FP32).
 * order_dev: NULL (rows in order every epoch) or epochs x n int32 row
 * indices (device); each epoch takes n / batch minibatches of consecutive
 * entries.  loss_hist_host: NULL or room for epochs * (n / batch) doubles
 * (minibatch losses).  Synchronises `stream`; ENUMERIC if training
 * diverges. */
int sl7_train(sl7_mlp* H, const sl7_train_spec* spec, const float* X_dev,
              const float* Y_dev, int64_t n, const int32_t* order_dev,
              double* loss_hist_host, void* stream);

/* Gradient of the loss over the B rows (one minibatch) with respect to the
 * parameter vector (same layout as the parameters) into grad_dev (FP32,
 * device); loss_host: NULL or the loss.  Synchronises `stream`.
 * This is the training step's weight gradient as its own call: with
 * sl7_train (whole epochs, Adam in place) it replaces a single-step train
 * call, leaving the optimiser of a single step to the caller (the Python
 * binding's SL7TrainLoss feeds it to torch.autograd).  The same weight
 * gradient is why sl7_adjoint has no weight-gradient output: the network's
 * parameters enter training through this loss, not through E[f(Y_T)]. */
int sl7_train_grad(const sl7_mlp* H, const float* X_dev, const float* Y_dev, int64_t B,
                   float* grad_dev, double* loss_host, void* stream);

/* --- launch plans ------------------------------------------------------ */
/* The plan a call uses when it is given none, for a launch of n_blocks
 * 64-path blocks (the sum of ceil(N / 64) over its instances) on a device
 * with n_cu compute units.  Host only, no device needed.  The split modes
 * take 12-wave workgroups (all weights in LDS) from 64 blocks per compute
 * unit, 4-wave ones below.  SL7_EINVAL for an unknown precision, n_cu < 1
 * or out == NULL. */
int sl7_default_plan(int prec, int64_t n_blocks, int n_cu, sl7_plan* out);

/* --- launch-plan autotuner -------------------------------------------- */
/* Times candidate plans on `shape` (a problem, N may be reduced) and
 * returns the fastest in *out; when cache_path is not NULL the result is
 * stored there as one JSON line per (arch, prec, d_in, m) key and read back
 * on later calls instead of re-timing. */
int sl7_autotune(const sl7_problem* shape, const sl7_mlp* H, int prec,
                 const char* cache_path, sl7_plan* out, void* stream);

/* The same for a batch: times each candidate plan on the n instances of
 * prs[] themselves, one persistent launch as sl7_simulate_batched makes it
 * (arguments checked as there), and returns the fastest in *out.  The cache
 * key adds a hash of the instances' shapes (model, m, M, N of each, in
 * order).  Synchronises `stream`. */
int sl7_autotune_batched(const sl7_problem* prs, int n, const sl7_mlp* H, int prec,
                         const char* cache_path, sl7_plan* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SL7_H */
