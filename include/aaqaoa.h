/*
 * aaqaoa.h -- C ABI of the MI355X (gfx950) MaxCut-QAOA statevector estimator.
 *
 * The library evaluates the p-layer QAOA state
 *     |psi(gamma, beta)> = prod_{l=1..p} e^{-i beta_l H_M} e^{-i gamma_l H_C} |+>^n
 * (QAOA section, eq. for |psi>_p; layer 1 is applied first and the cost unitary
 * precedes the mixer in every layer, as written out in eq. A2), with the unweighted
 * MaxCut Hamiltonian H_C = 1/2 sum_{(i,j) in E} (1 - Z_i Z_j) and the mixer
 * H_M = sum_i X_i, and returns the expectation of either
 *     H_C                                                      (AAQ_OBS_HC), or
 *     H_red = 1/2 sum_m |S_m| (1 - Z_{i_m} Z_{j_m})            (AAQ_OBS_HRED)
 * where (i_m, j_m) is a representative edge of Aut(G) edge orbit S_m ("Reducing
 * the Hamiltonian" section).  On the Aut(G)-invariant QAOA state both are equal
 * (Eq. exact); the library does not check that the supplied orbits are real
 * Aut(G) orbits -- a wrong orbit list silently breaks that identity.  Use
 * AAQ_AGG_PER_TERM with AAQ_OBS_HC to inspect per-edge <Z_i Z_j> within orbits.
 *
 * Conventions
 *   - vertex v = qubit v = bit v of the amplitude index z (little-endian);
 *   - gamma[l], beta[l] in radians, l = 0..p-1, l = 0 applied first;
 *   - energies are <H> including the constant (the expected cut value, >= 0);
 *   - the cost layer multiplies amplitude z by exp(-i gamma C(z)), C(z) = number
 *     of cut edges (an exact integer), with gamma*C(z) reduced in FP64;
 *   - amplitudes are complex64 (interleaved float re/im, 8 bytes) unless the call
 *     asks for AAQ_PREC_C128 (complex128, 16 bytes); expectation and gradient
 *     accumulations are FP64.
 *
 * Memory ownership
 *   - Host arrays passed in are only read during the call.
 *   - Device buffers (state, lambda, workspace, device outputs) are owned by the
 *     caller.  The library never allocates device memory.
 *   - Calls that return results through host pointers synchronise the stream.
 *   - aaq_plan objects are host objects owned by the library (aaq_plan_destroy).
 *
 * Errors
 *   Every entry point returns an aaq_status.  Arguments are validated on the host
 *   before any HIP call; on error the outputs are left untouched and
 *   aaq_last_error_message() (thread-local) explains the failure.  Nothing aborts.
 */
#ifndef AAQAOA_H
#define AAQAOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AAQ_OK = 0,
  AAQ_ERR_INVALID_ARG = 1, /* null pointer, bad enum, bad p or n               */
  AAQ_ERR_GRAPH = 2,       /* vertex out of range, self-loop, duplicate edge   */
  AAQ_ERR_ORBITS = 3,      /* orbit sizes do not sum to |E|, bad representative */
  AAQ_ERR_PARAMS = 4,      /* non-finite gamma or beta                         */
  AAQ_ERR_BUFFER = 5,      /* state / lambda / workspace buffer too small      */
  AAQ_ERR_UNSUPPORTED = 6, /* valid request the library does not support       */
  AAQ_ERR_HIP = 7          /* a HIP runtime call failed                        */
} aaq_status;

/* The selector arguments below are plain 32-bit integers with named values, so any value
 * a caller passes is well defined and is checked (AAQ_ERR_INVALID_ARG when unknown). */
typedef int32_t aaq_observable;
enum { AAQ_OBS_HC = 0, AAQ_OBS_HRED = 1 };

/* How the expectation is aggregated (estimator cost section):
 *   FUSED          -- one integer h(z) per amplitude, one pass (default);
 *   PER_TERM       -- one <Z_i Z_j> accumulator per observable term in the same pass,
 *                     energy = sum_t (w_t/2)(1 - <ZZ>_t); fills zz_out;
 *   PASS_PER_TERM  -- the final state is written and every term's <Z_i Z_j> is a
 *                     separate O(2^n) pass over it (the per-term estimator structure
 *                     the paper describes; its cost grows with the number of terms). */
typedef int32_t aaq_aggregation;
enum { AAQ_AGG_FUSED = 0, AAQ_AGG_PER_TERM = 1, AAQ_AGG_PASS_PER_TERM = 2 };

typedef int32_t aaq_precision;
enum { AAQ_PREC_C64 = 0, AAQ_PREC_C128 = 1 };

/* A MaxCut instance with its Aut(G) edge orbits (Algorithm 1 output).
 *   n           qubits = vertices, 1 <= n <= 34
 *   num_edges   |E| >= 0 (n = 1 requires 0)
 *   edges       [2*|E|] pairs (u, v), 0 <= u, v < n, u != v, no duplicate edge
 *   num_orbits  |O_E| (0 iff |E| = 0)
 *   orbit_rep   [|O_E|] edge index of each orbit's representative (0 <= . < |E|)
 *   orbit_size  [|O_E|] |S_m| >= 1, summing to |E|
 *   edge_orbit  [|E|] orbit id of every edge, or NULL; when given, the library
 *               checks that sizes and representatives agree with it.
 *   edge_weight [|E|] integer edge weights w_ij >= 1 of the MaxCut H_P (the QAOA
 *               section's H_P = 1/2 sum w_ij (1 - Z_i Z_j); the paper's experiments use
 *               w = 1), or NULL for all 1.  The cut C(z) = sum w_ij [z_i != z_j] stays an
 *               exact integer; the total weight sum w_ij must be <= AAQ_MAX_COST (the
 *               phase tables hold C = 0 .. sum w).  The orbits must be orbits of the
 *               weight-preserving automorphisms (aaq_edge_orbits with the same weights);
 *               with edge_orbit given, equal weights inside every orbit are checked.
 *               H_C's terms carry w_ij, H_red's the orbit size times the
 *               representative's weight.  Single-instance evaluations of weighted
 *               instances run weighted copies of the specialised sweeps (the cut taken
 *               from per-set cost-term lists); weighted plan units and light cones run
 *               the sweeps whose steps are taken from the sweep program at run time. */
#define AAQ_MAX_COST 561
typedef struct {
  int32_t n;
  int32_t num_edges;
  const int32_t *edges;
  int32_t num_orbits;
  const int32_t *orbit_rep;
  const int32_t *orbit_size;
  const int32_t *edge_orbit;
  const int32_t *edge_weight;
} aaq_problem;

/* Host-side validation of a problem and depth p (1 <= p <= AAQ_MAX_P). No HIP calls. */
#define AAQ_MAX_P 64
#define AAQ_MAX_N 34
aaq_status aaq_validate(const aaq_problem *prob, int p);

/* Bytes of one state buffer (2^n amplitudes) at the given precision. */
aaq_status aaq_state_bytes(const aaq_problem *prob, aaq_precision prec, size_t *bytes);

/* Workspace bytes needed by aaq_energy / aaq_energy_grad for this problem, depth,
 * gradient flag, observable, aggregation and precision. */
aaq_status aaq_workspace_size(const aaq_problem *prob, int p, int with_grad, aaq_observable obs,
                              aaq_aggregation agg, aaq_precision prec, size_t *bytes);

/* <H> of the QAOA state (F_p, QAOA section; aggregation eq. of the estimator-cost
 * section; H_red as in "Reducing the Hamiltonian").
 *   d_state      device buffer of >= aaq_state_bytes; overwritten (it holds intermediate
 *                states; its final contents are unspecified)
 *   d_ws         device workspace of >= aaq_workspace_size bytes
 *   stream       hipStream_t (NULL = default stream)
 *   energy_out   host double
 *   zz_out       host double[T] (T = |E| for H_C, |O_E| for H_red) or NULL; filled
 *                only for PER_TERM and PASS_PER_TERM aggregation
 *   norm_out     host double <psi|psi> (diagnostic) or NULL */
aaq_status aaq_energy(const aaq_problem *prob, int p, const double *gamma, const double *beta,
                      aaq_observable obs, aaq_aggregation agg, aaq_precision prec, void *d_state,
                      size_t state_bytes, void *d_ws, size_t ws_bytes, void *stream, double *energy_out,
                      double *zz_out, double *norm_out);

/* <H> and its gradient by the adjoint method: dE/dtheta = 2 Im <lambda|G|psi> for each
 * gate e^{-i theta G} (G = H_C for gamma_l, G = sum_q X_q for beta_l), with lambda the
 * observable applied to the final state and swept backwards with psi; the gates are
 * unitary, so psi is uncomputed on the way back and no checkpoints are kept.
 *   d_lambda     second device buffer of >= aaq_state_bytes
 *   dgamma_out, dbeta_out  host double[p] */
aaq_status aaq_energy_grad(const aaq_problem *prob, int p, const double *gamma, const double *beta,
                           aaq_observable obs, aaq_precision prec, void *d_state, size_t state_bytes,
                           void *d_lambda, size_t lambda_bytes, void *d_ws, size_t ws_bytes, void *stream,
                           double *energy_out, double *dgamma_out, double *dbeta_out, double *norm_out);

/* Forward-state checkpoints (memory for bandwidth): aaq_energy_grad_checkpointed computes
 * the same energy and gradient as aaq_energy_grad (up to floating-point summation order),
 * but every forward sweep keeps its output state in its own slot of d_ckpt, so each
 * backward sweep reads psi from there instead of uncomputing it and writing it back: one
 * state pass fewer per backward sweep.  d_ckpt needs aaq_checkpoint_bytes (a few states;
 * 8 x 512 MiB at n = 26, p = 4); d_lambda, d_ws and the outputs are as for
 * aaq_energy_grad.  Problems whose state is one tile (n <= 13) need one state. */
aaq_status aaq_checkpoint_bytes(const aaq_problem *prob, int p, aaq_precision prec, size_t *bytes);
aaq_status aaq_energy_grad_checkpointed(const aaq_problem *prob, int p, const double *gamma, const double *beta,
                                        aaq_observable obs, aaq_precision prec, void *d_ckpt, size_t ckpt_bytes,
                                        void *d_lambda, size_t lambda_bytes, void *d_ws, size_t ws_bytes,
                                        void *stream, double *energy_out, double *dgamma_out, double *dbeta_out,
                                        double *norm_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same energy and adjoint gradient as
 * aaq_energy_grad, bit for bit, with the workspace taken from a static device array of
 * AAQ_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends (its device address is looked up once per device).  The call allocates
 * no device memory and no pinned host memory: the upload goes through ordinary host
 * memory, so the call synchronises the stream like aaq_energy_grad.
 *   d_state, d_lambda  caller buffers as for aaq_energy_grad
 *   returns AAQ_ERR_BUFFER before any HIP call when the problem's workspace
 *   (aaq_workspace_size with gradients) exceeds AAQ_NOALLOC_SCRATCH_BYTES.
 * Every call on one GPU uses that GPU's array: calls that overlap in time on one GPU
 * (several host threads or streams) race and must be serialised by the caller. */
#define AAQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
aaq_status aaq_energy_grad_noalloc(const aaq_problem *prob, int p, const double *gamma, const double *beta,
                                   aaq_observable obs, aaq_precision prec, void *d_state, size_t state_bytes,
                                   void *d_lambda, size_t lambda_bytes, void *stream, double *energy_out,
                                   double *dgamma_out, double *dbeta_out, double *norm_out);

/* Exact integer values of the observable's diagonal for every z in [0, 2^n):
 * C(z) for AAQ_OBS_HC, h_red(z) = sum_m |S_m| [z_{i_m} != z_{j_m}] for AAQ_OBS_HRED
 * (the diagonal of H_C and H_red without the 1/2 (1 - ZZ) rewriting), computed by the
 * same device code that the cost layer and the expectation use.
 *   d_ws   device workspace of >= 512 + 16 * T * (1 + 2 * aaq_num_sets(n, prec)) bytes
 *          (T = number of observable terms: the graph block and the term lists)
 *   d_out  device int32[2^n] (16 GiB at n = 32, 64 GiB at n = 34).  Synchronises the stream. */
aaq_status aaq_cut_values(const aaq_problem *prob, aaq_observable obs, void *d_ws, size_t ws_bytes, int32_t *d_out,
                          void *stream);

/* Diagnostic variant: the values as computed inside tile set `set_index`
 * (0 .. aaq_num_sets(n, prec) - 1) at register arrangement 0 (the load/store layout)
 * or 1 (the layout where the cost phase is applied).  Every variant must equal
 * aaq_cut_values bit for bit. */
aaq_status aaq_cut_values_layout(const aaq_problem *prob, aaq_observable obs, int set_index, int arrangement,
                                 aaq_precision prec, void *d_ws, size_t ws_bytes, int32_t *d_out, void *stream);

/* Number of tile sets (groups of qubits mixed in one sweep) that the built-in tile-size
 * rule gives for n qubits: 1 when the whole state is one tile (n <= 13); the
 * diagnostic aaq_cut_values_layout uses the same rule.  Precision does not change it. */
int aaq_num_sets(int n, aaq_precision prec);

/* ---------------------------------------------------------------- tile size and autotuning
 * The sweeps process the state in tiles of 2^12 or 2^13 amplitudes per workgroup (256 or
 * 512 threads).  By default the size that gives the fewest sweeps is used, 12 on ties.
 * aaq_set_tile_bits overrides the choice for one (n, precision, gradient) class of calls
 * (0 restores the default); the setting is process-wide and guarded by a mutex.
 * aaq_autotune times `reps` calls of aaq_energy (with_grad = 0) or aaq_energy_grad
 * (with_grad = 1) at each tile size with the caller's buffers (as for those calls;
 * d_lambda may be NULL without gradients), keeps the faster one for the problem's class
 * and reports it; ms_per_call, if not NULL, receives the two timings (tile 12, tile 13).
 * These calls choose launch shapes only (not a step of the paper's method): results
 * differ between tile sizes by floating-point summation order at most. */
aaq_status aaq_set_tile_bits(int n, aaq_precision prec, int with_grad, int tile_bits);
int aaq_get_tile_bits(int n, aaq_precision prec, int with_grad);
aaq_status aaq_autotune(const aaq_problem *prob, int p, int with_grad, aaq_observable obs, aaq_precision prec,
                        void *d_state, size_t state_bytes, void *d_lambda, size_t lambda_bytes, void *d_ws,
                        size_t ws_bytes, void *stream, int reps, int *best_tile_bits, double *ms_per_call);

/* ---------------------------------------------------------------- batched plans
 * Many (instance, parameter point) units evaluated together.  Units whose state fits
 * one tile (n <= 13) run in a persistent kernel: each workgroup takes the next unit from
 * a device work counter (largest n first) and runs its whole forward (and backward)
 * sweep sequence in registers, one launch per tile size.  Larger units are grouped by
 * tile size and tile-set count, and each sweep step is one launch over every tile of
 * every unit of the group; the persistent small-unit launches run concurrently with
 * that chain (a second stream, a fork and a join in the captured graph; with
 * small_streams each of them on a stream of its own).  Units with n > 13 store and sweep
 * the half state (the spin-flip symmetry, as for the single-instance calls, when
 * aaq_set_half_state allows it) and, with gradients, keep their forward states.  With
 * single_launch every unit runs in the persistent kernel (a large unit is swept tile by
 * tile by the one workgroup that takes it), so the whole batch is one launch after the
 * phase tables.  Replays are captured once in a HIP graph.
 *   probs[count]  the instance of every unit (the same instance may repeat)
 *   d_params      device double[count][2p]: gamma_0..gamma_{p-1}, beta_0..beta_{p-1}
 *   d_out         device double[count][2 + 2p]: energy, norm, dE/dgamma[p], dE/dbeta[p]
 *                 (gradients only when with_grad) */
typedef struct aaq_plan aaq_plan;

typedef struct {
  int use_graph;      /* capture the launches in a HIP graph and replay it (default 1) */
  int workgroups;     /* persistent workgroups per unit-kernel launch; 0 = automatic */
  int sort_units;     /* 1 = largest n first (default) */
  aaq_precision prec; /* amplitude precision (default AAQ_PREC_C64) */
  int tile_bits_large;     /* tile size (log2 amplitudes per workgroup tile: 12 or 13) of the units
                              with n > 13; 0 = fewest sweeps, then 12 (default) */
  int min_tile_bits_small; /* units with n <= 13 run on the smallest compiled tile (10, 12 or 13
                              amplitude bits) that is >= max(n, this); 0 = 10 (default) */
  int single_launch;       /* 1 = every unit in the persistent kernel (one launch per tile size);
                              0 = units with n > 13 as batched sweep steps (default) */
  int small_streams;       /* 1 = each persistent small-unit launch (one per tile size) on a stream
                              of its own, concurrent with the others; 0 = all of them on one
                              stream beside the batched sweep steps (default) */
  int max_small_n;         /* units with n <= this run in the persistent small-unit kernel, the
                              others as batched sweep steps (13, or 12: 13-qubit units then take
                              two 12-bit tiles); 0 = 12 when some unit has n > 13 and
                              single_launch is 0 (the steps run anyway), else 13 (default) */
} aaq_plan_opts;

/* Fills opts with the defaults above. */
void aaq_plan_default_opts(aaq_plan_opts *opts);

aaq_status aaq_plan_workspace_size(const aaq_problem *probs, int count, int p, aaq_observable obs, int with_grad,
                                   const aaq_plan_opts *opts, size_t *bytes);

/* Validates every unit, lays out the workspace (descriptors, phase tables, per-unit
 * state buffers for n > 13: with gradients the forward state after each of a unit's
 * forward sweep steps, when there are at most 32 of them, and lambda; psi and lambda
 * otherwise) and uploads descriptors on `stream`. */
aaq_status aaq_plan_create(const aaq_problem *probs, int count, int p, aaq_observable obs, int with_grad,
                           const aaq_plan_opts *opts, void *d_ws, size_t ws_bytes, void *stream,
                           aaq_plan **out);

/* Asynchronous on `stream`: reads parameters from d_params, writes d_out.  With
 * use_graph the first call (or a call with new buffer addresses) captures a graph
 * and later calls replay it. */
aaq_status aaq_plan_execute(aaq_plan *plan, const double *d_params, double *d_out, void *stream);

void aaq_plan_destroy(aaq_plan *plan);

/* Plan autotuner: builds the plan with every candidate of tile_bits_large (12, 13; when
 * some unit has n > 13), min_tile_bits_small (10, 12, 13; when some unit has n <= 12),
 * workgroups (automatic, one and four per compute unit; when some unit has n <= 13) and
 * single_launch (0, 1; when some unit has n > 13), small_streams (0, 1; when some unit has
 * n <= 13) and max_small_n (13, 12; when some unit has n = 13 and some n > 13) on top of
 * `base` (NULL = defaults),
 * times `reps` executions of each with HIP
 * events on `stream` (after one warm-up execution) and returns the fastest options in
 * *best and their time per execution in *best_ms (may be NULL).  Candidates whose
 * workspace exceeds ws_bytes are skipped.  d_params / d_out as for aaq_plan_execute;
 * d_out is overwritten.  Synchronises the stream. */
aaq_status aaq_plan_autotune(const aaq_problem *probs, int count, int p, aaq_observable obs, int with_grad,
                             const aaq_plan_opts *base, void *d_ws, size_t ws_bytes, const double *d_params,
                             double *d_out, void *stream, int reps, aaq_plan_opts *best, double *best_ms);

/* ---------------------------------------------------------------- resident evaluator
 * For optimizer loops whose parameters live on the device (e.g. a torch optimizer on the
 * GPU): the same fused evaluation as aaq_energy / aaq_energy_grad(_checkpointed), with the
 * instance, its sweep programs and tile sets uploaded once at creation.  Each execute
 * reads d_params = [gamma[p], beta[p]] (device doubles) and writes d_out = [energy, norm,
 * dgamma[p], dbeta[p]] (device doubles; the gradient entries are 0 without with_grad),
 * asynchronously on the stream: no host synchronisation and no host-device copy, so
 * evaluations queue back to back.
 *   with_grad   energy + adjoint gradient
 *   checkpoint  forward-state checkpoints (with_grad only): d_state then holds the
 *               checkpoint states
 *   d_state, d_lambda, d_ws  caller buffers of at least the sizes from
 *               aaq_resident_workspace_size (state_bytes also bounds d_lambda with
 *               with_grad, one state); they stay owned by the caller, must outlive the
 *               evaluator and are used by every execute, so executions on one evaluator
 *               are to be ordered on one stream.
 * Create validates like aaq_energy and synchronises the stream once (the upload);
 * execute checks only its pointers. */
typedef struct aaq_resident aaq_resident;
aaq_status aaq_resident_workspace_size(const aaq_problem *prob, int p, aaq_observable obs, int with_grad, int checkpoint,
                                       aaq_precision prec, size_t *ws_bytes, size_t *state_bytes);
aaq_status aaq_resident_create(const aaq_problem *prob, int p, aaq_observable obs, int with_grad, int checkpoint,
                               aaq_precision prec, void *d_state, size_t state_bytes, void *d_lambda,
                               size_t lambda_bytes, void *d_ws, size_t ws_bytes, void *stream, aaq_resident **out);
aaq_status aaq_resident_execute(aaq_resident *r, const double *d_params, double *d_out, void *stream);
void aaq_resident_destroy(aaq_resident *r);

/* ---------------------------------------------------------------- half state
 * MaxCut QAOA states are invariant under flipping every bit (|+>, the cut phase and the
 * mixer all commute with the global flip; so are h and lambda = (h - c) psi), so the single-
 * instance and resident evaluations store and sweep only the amplitudes with bit n-1 = 0
 * and double every sum (the same results up to rounding order, half the state traffic
 * and half the vector work).  Used when the program has at least two tile sets, the state
 * is not of the one size whose 2^n amplitudes exceed 4 GiB while their half does not (n = 30
 * complex64, n = 29 complex128: those keep the full state), and the call neither keeps the
 * final state (sampling) nor passes over it per term.  On by
 * default; the switch is process-wide and takes effect at the next call (it is part of
 * the cached host plan's key).  State buffers sized by aaq_state_bytes stay valid. */
void aaq_set_half_state(int enable);
int aaq_get_half_state(void);

/* ---------------------------------------------------------------- final-state sampling
 * The read-out the paper's approximation ratios come from: bitstrings z drawn with
 * probability |psi(z)|^2 from the depth-p QAOA state (its results section samples the
 * final state), their cut values and the best and mean cut.  The forward sweeps keep the
 * final state in d_state; each shot k takes the uniform number u_k = d_uniform[k] (values
 * outside [0, 1) are clamped into it, NaN reads as 0) and returns the smallest bitstring z, in the order
 * of the integers z, whose cumulative probability exceeds u_k (inverse CDF, FP64
 * accumulation of the complex64 or complex128 probabilities).  Random numbers are the
 * caller's: the same u gives the same shots.
 *   d_uniform  device double[num_shots]
 *   d_samples  device uint64[num_shots]: bit v of sample k = vertex v's side
 *   d_cuts     device int32[num_shots]: cut value C(z) of each sample (exact integers)
 *   best_cut_out, mean_cut_out  host doubles (may be NULL)
 * d_state as for aaq_energy; the workspace from aaq_sample_workspace_size.  Synchronises
 * the stream; AAQ_ERR_UNSUPPORTED for a graph without edges. */
aaq_status aaq_sample_workspace_size(const aaq_problem *prob, int p, aaq_precision prec, size_t *bytes);
aaq_status aaq_sample(const aaq_problem *prob, int p, const double *gamma, const double *beta, aaq_precision prec,
                      int num_shots, const double *d_uniform, void *d_state, size_t state_bytes, void *d_ws,
                      size_t ws_bytes, void *stream, uint64_t *d_samples, int32_t *d_cuts, double *best_cut_out,
                      double *mean_cut_out);

/* ---------------------------------------------------------------- edge orbits
 * Edge orbits of Aut(G) on the host (the paper's Algorithm 1 with its generator source,
 * nauty in the paper, replaced by an individualisation-refinement search): the edge list
 * is closed under automorphism generators by breadth-first search, each class seeded at
 * its lowest-index edge (with a sorted edge list, exactly Algorithm 1's order); whenever
 * two classes whose seed edges have equal colour-refinement invariants are apart, the
 * search looks for an automorphism mapping one seed onto the other.  The result is the
 * orbit partition under the whole group Aut(G).
 *   edges       [2 * num_edges] (u, v) pairs, any order; 0 <= u, v < n, u != v, no duplicates
 *   edge_weight [num_edges] integer weights, or NULL: with weights the group is the
 *               weight-preserving automorphisms (refinement sees edge weights, a
 *               generator maps every edge onto one of equal weight)
 *   orbit_of    out [num_edges]: class of each edge
 *   num_orbits  out: number of classes
 *   orbit_rep   out [num_edges] (first *num_orbits used): seed edge index of each class
 *   orbit_size  out [num_edges] (first *num_orbits used): class sizes
 * The outputs fill an aaq_problem's orbit arrays directly.  Host only, n <= 4096; errors
 * AAQ_ERR_GRAPH / AAQ_ERR_INVALID_ARG, outputs untouched on error.  The search is
 * exponential in the worst case (as is any generator search), fast on the graph families
 * of the paper. */
aaq_status aaq_edge_orbits(int n, int num_edges, const int32_t *edges, const int32_t *edge_weight, int32_t *orbit_of,
                           int32_t *num_orbits, int32_t *orbit_rep, int32_t *orbit_size);

/* The structural descriptor of combined-RCC coverage (the paper's subsection of that name,
 * Eq. for eta_p):  eta_p = 1 - |U_{e in R} RCC_p(e)| / |E|, the fraction of edges outside
 * the union of the representatives' reverse causal cones.  RCC_p(e) of e = (i, j) is the
 * set of cost gates that do not commute through to Z_i Z_j in p layers: the edges with an
 * endpoint within graph distance p - 1 of {i, j}; the cone's qubits are the vertices within
 * distance p.
 *   edges        [2 * num_edges] (u, v) pairs, validated as in aaq_edge_orbits; 1 <= |E| <= 65536
 *   orbit_of     [num_edges] orbit id of each edge, 0 .. num_orbits - 1 (aaq_edge_orbits output)
 *   rep          [num_orbits] representative edge of each orbit (an edge of that orbit), or
 *                NULL: eta_out is then the exact mean over representatives drawn uniformly
 *                and independently in every orbit (the tables' random selection)
 *   p            >= 1
 *   eta_out      out: eta_p
 *   qubit_elim_out  out or NULL: the qubit-elimination fraction shown beside eta_1 in the
 *                paper's figure of structural descriptors, read as the share of the n qubits
 *                outside the union of the cones' qubits (mean over the random choice when
 *                rep is NULL)
 *   vertex_cover_out  [n] or NULL (only with rep): 1 for every qubit of the union of the
 *                cones, else 0
 * Host only, O(|E| (n + |E|)); errors AAQ_ERR_INVALID_ARG / AAQ_ERR_GRAPH / AAQ_ERR_ORBITS,
 * outputs untouched on error. */
aaq_status aaq_rcc_eta(int n, int num_edges, const int32_t *edges, const int32_t *orbit_of, int num_orbits,
                       const int32_t *rep, int p, double *eta_out, double *qubit_elim_out,
                       uint8_t *vertex_cover_out);

/* ---------------------------------------------------------------- light cones
 * Light-cone evaluation, the locality reduction the paper names as compounding with the
 * orbit reduction (its discussion of reverse causal cones): the depth-p expectation of a
 * term Z_i Z_j depends only on the subgraph induced by the vertices within distance p of
 * {i, j}, exactly.  Each term of the observable (H_C: every edge, weight 1; H_red: one
 * representative per edge orbit, weight = orbit size) is simulated on its own cone as one
 * unit of a batched plan (the kernels above), and
 *   <H> = sum_t (w_t / 2) (1 - <Z_i Z_j>_t)
 * together with its gradient are the sums over the units.  Cones are built on the host by
 * breadth-first search; vertices keep their order, relabelled 0..|cone|-1.
 *   d_params  device double[2p]: gamma_0..gamma_{p-1}, beta_0..beta_{p-1}
 *   d_out     device double[2 + 2p]: energy, mean norm of the unit states, dE/dgamma[p],
 *             dE/dbeta[p] (gradients only when with_grad)
 * Errors as for the plans; AAQ_ERR_UNSUPPORTED for a graph without edges.  The handle
 * owns its unit descriptions; the workspace is the caller's. */
typedef struct aaq_lightcone aaq_lightcone;

/* Host only: number of units (terms), the largest cone (qubits) and the total number of
 * amplitudes of all cone states (sum over units of 2^|cone|). */
aaq_status aaq_lightcone_info(const aaq_problem *prob, int p, aaq_observable obs, int *units, int *max_qubits,
                              double *amplitudes);
aaq_status aaq_lightcone_workspace_size(const aaq_problem *prob, int p, aaq_observable obs, int with_grad,
                                        const aaq_plan_opts *opts, size_t *bytes);
/* Builds the cones and their plan (opts as for aaq_plan_create) and uploads it on `stream`. */
aaq_status aaq_lightcone_create(const aaq_problem *prob, int p, aaq_observable obs, int with_grad,
                                const aaq_plan_opts *opts, void *d_ws, size_t ws_bytes, void *stream,
                                aaq_lightcone **out);
/* Asynchronous on `stream`; with opts.use_graph the launches are captured once per
 * (d_params, d_out, stream) and replayed. */
aaq_status aaq_lightcone_execute(aaq_lightcone *lc, const double *d_params, double *d_out, void *stream);
void aaq_lightcone_destroy(aaq_lightcone *lc);

/* ---------------------------------------------------------------- diagnostics */
/* Per-kernel timing.  While enabled, every kernel launch of the library (outside a
 * stream capture, of the classes selected by aaq_timing_classes) carries two HIP events in its dispatch on the stream it is launched
 * on (the kernel's start and end; a launch of two kernels is timed from the first's
 * start to the second's end); aaq_timing_read waits for the events and returns, per
 * kernel class ("sweep_1state", "sweep_2state", "tables", "reduce", "zz_pass",
 * "units"), the launch count, the summed event time and the algorithmic bytes of the
 * state buffers the launches read and write.  For measurement only: it creates two
 * events per launch. */
typedef struct {
  char name[32];
  long long launches;
  double total_ms;
  double bytes;
} aaq_kernel_timing;
aaq_status aaq_timing_enable(int on);
aaq_status aaq_timing_read(aaq_kernel_timing *out, int max, int *count, int reset);
/* The kernel classes whose launches carry events while timing is on, as a bit mask in the
 * order listed above (bit 0 "sweep_1state", 1 "sweep_2state", 2 "tables", 3 "reduce",
 * 4 "zz_pass", 5 "units"); every class (63) until changed.  Launches of the other classes
 * run without events and are not counted.  AAQ_ERR_INVALID_ARG for a negative mask or
 * one with bits above 5 (the selection is then unchanged). */
aaq_status aaq_timing_classes(int mask);

const char *aaq_status_string(aaq_status s);
const char *aaq_last_error_message(void);

/* Library version string, e.g. "aaqaoa 0.1 gfx950". */
const char *aaq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AAQAOA_H */
