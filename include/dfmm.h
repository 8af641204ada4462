/*
 * dfmm.h -- C ABI of libdfmm, a gfx950 (MI355X) implementation of the
 * kernel-independent Lagrange fast multipole method for the stress and
 * Peach-Koehler forces of straight dislocation segments in isotropic and
 * cubic-anisotropic elastic media (Chen, Aubry, Oppelstrup, Arsenlis, Darve,
 * "Fast algorithms for evaluating the stress field of dislocation lines in
 * anisotropic elastic media").
 *
 * What is computed (Sec. 2, Eqs. stress, kernel, stress_discrete, stress3):
 *   every segment i (end points x1, x2, Burgers vector b) carries n_quad
 *   Gauss-Legendre points y_ik = x1 + (1+u_k)/2 (x2-x1) with strengths
 *   q_ik = (omega_k/2) b (x) (x2-x1).  The stress at every point is
 *   s(x) = sum over all points j of K(x - y_j) q_j, with the 54-component kernel
 *   K = -eps C C dG (the sign makes a straight dislocation's stress the
 *   textbook one) and the non-singular Green's-function derivative dG with
 *   core radius a.  The force at the two ends of each segment is the Gauss
 *   quadrature of (sigma.b) x (x2-x1) with linear shape functions.
 *   dfmm_fmm_forces evaluates the sum with the Lagrange FMM (Sec. 4,
 *   Alg. lagrange): P2M, M2M, M2L (FFT-diagonal block-Toeplitz product,
 *   Theorem 1), L2L, L2P and the direct near field over the 27 neighbour
 *   leaves.  dfmm_direct_forces evaluates the same sum directly.
 *
 * Conventions:
 *   - Memory: every array argument marked "device" is a device pointer on
 *     the current HIP device, owned by the caller.  seg is [n_seg][2][3]
 *     double (x1 then x2), burgers [n_seg][3] double, forces [n][2][3]
 *     double (force on end 1 then end 2).  The library owns plans, trees
 *     and their workspaces.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  All device work of a call is ordered on that stream.
 *   - Errors: every entry point returns a dfmm_status; nothing is thrown
 *     across the ABI.  dfmm_last_error() gives a thread-local message for
 *     the last failing call.  On failure no output is guaranteed.
 *   - Threads: a plan is read-only after dfmm_fmm_setup and may be shared
 *     by concurrent calls, except that the surrogate calls that change its
 *     network or switch it (dfmm_surrogate_train, _use, _set_params, _load)
 *     modify the plan and must not overlap any other call using it; a tree
 *     belongs to one stream at a time.
 */
#ifndef DFMM_H
#define DFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DFMM_OK = 0,
  DFMM_E_ARG = -1,        /* invalid argument (null pointer, size, range)       */
  DFMM_E_NOMEM = -2,      /* device or host allocation failed                   */
  DFMM_E_HIP = -3,        /* a HIP runtime call or kernel launch failed          */
  DFMM_E_OUT_OF_BOX = -4, /* a quadrature point lies outside the root cube       */
  DFMM_E_NONFINITE = -5,  /* a segment coordinate is NaN or infinite             */
  DFMM_E_STATE = -6       /* objects that do not belong together (plan/tree)     */
} dfmm_status;

/* Arithmetic of the evaluation (the operators are always precomputed in
 * double precision).  DFMM_MIXED_F16 is DFMM_MIXED with the M2L Hadamard
 * product taking f16 operands (operator spectra and source spectra, each
 * level scaled into f16's range) with f32 accumulation. */
enum { DFMM_FP64 = 0, DFMM_MIXED = 1, DFMM_MIXED_F16 = 2 };
/* M2L operator store (Eq. mem_unif and the symmetry reduction of Sec. 6):
 * DFMM_M2L_FFT keeps the spectra of the 158 canonical offsets (one of each
 * pair o, -o of the 316; the kernel is odd); DFMM_M2L_FFT_SYM keeps only the
 * 16 offsets that represent the classes of the 316 under the 48 reflections
 * and axis permutations of the cube (which leave a cubic or isotropic medium
 * unchanged) and expands them in the M2L product: about a tenth of the
 * memory and a quarter of the precompute's kernel evaluations. */
enum { DFMM_M2L_FFT = 0, DFMM_M2L_FFT_SYM = 1 };
/* Anisotropic kernel: DFMM_KERNEL_EXACT is the unit-circle quadrature;
 * DFMM_KERNEL_SURROGATE trains the library's network at setup (default
 * configuration, dfmm_surrogate_default_cfg) and uses it wherever its
 * residual gate passes, the exact quadrature elsewhere (see the surrogate
 * calls below).  Ignored for isotropic media (closed form). */
enum { DFMM_KERNEL_EXACT = 0, DFMM_KERNEL_SURROGATE = 1 };

typedef struct dfmm_plan dfmm_plan; /* medium, order, depth, M2L spectra        */
typedef struct dfmm_tree dfmm_tree; /* sorted points, cells, lists, workspaces   */

typedef struct {
  int order;          /* p: interpolation nodes per dimension, 2..8 (Sec. 4.1;
                         the paper's "p-th order" interpolant has p^3 nodes)     */
  int depth;          /* D: leaf level, 2..10; leaves are cells of side
                         box_size / 2^D; M2L runs on levels 2..D               */
  double c11, c12, c44; /* cubic stiffness in the crystal axes (= x, y, z).
                         Isotropic iff 2 c44 == c11 - c12 (to 1e-12 relative):
                         then the closed form of Eq. k_iso is used; otherwise
                         dG comes from unit-circle quadrature (n_circle points) */
  double core_a;      /* non-singular core radius a >= 0                         */
  double box_lo[3];   /* lower corner of the root cube                           */
  double box_size;    /* side of the root cube; every quadrature point must lie
                         in [box_lo, box_lo + box_size]^3                        */
  int n_quad;         /* Gauss-Legendre points per segment, 1..8 (usually 3)    */
  int n_circle;       /* unit-circle quadrature points, even, 8..256 (64)       */
  int precision;      /* DFMM_FP64: all arithmetic in double.
                         DFMM_MIXED: P2M..L2P and the near field in float with
                         float accumulation, near pairs closer than 2a in
                         double, far + near combined and forces in double.
                         DFMM_MIXED_F16: as DFMM_MIXED, the M2L product on
                         f16 operands with f32 accumulation                   */
  int m2l_mode;       /* DFMM_M2L_FFT or DFMM_M2L_FFT_SYM (operator store)       */
  int aniso_kernel;   /* DFMM_KERNEL_EXACT or DFMM_KERNEL_SURROGATE              */
  int lsq_degree;     /* 0: Lagrange interpolation on the p equispaced nodes
                         (degree p-1).  d in 1..p-1: the stabilised scheme of
                         Sec. 4.3, the least-squares polynomial of degree d
                         fitted to the node values (the M2L takes the fit's
                         node values of each W, and L2L/L2P those of each
                         local expansion; M2M and P2M stay Lagrange);
                         DFMM_LSQ_AUTO: the largest d < 2 sqrt(p), which is
                         p-1 (plain interpolation) for p < 6.  Degree p-1 is
                         run as 0.                                             */
  int leaf_max;       /* 0: uniform tree, every leaf on level `depth`.  n > 0:
                         adaptive tree (Sec. 3: the region is partitioned until
                         every leaf holds few segments): a cell above level
                         `depth` holding more than n quadrature points is
                         split, so leaves lie on several levels; the FMM then
                         adds the lists that join leaves of different levels
                         (direct sums with adjacent leaves of any level,
                         multipole weights of finer cells acting on a leaf's
                         points, points of coarser leaves acting on a cell's
                         nodes).  Requires lsq_degree 0 and the exact kernel. */
  int freq_chunks;    /* M2L spectra in chunks along the first frequency
                         axis (1..2p-1): a tree holds the source and target
                         spectra of one chunk of one level at a time, the
                         forward transform is repeated per chunk and the
                         inverse transforms are summed.  0: as few chunks as
                         keep them within half of the device memory free at
                         tree build.                                          */
} dfmm_params;
#define DFMM_LSQ_AUTO (-1)

/* Fill *p with defaults: order 5, depth 4, isotropic mu = 1, nu = 0.3,
 * a = 1e-3, root cube [-0.05, 1.05]^3, n_quad 3, n_circle 64, FP64,
 * DFMM_M2L_FFT, DFMM_KERNEL_EXACT, Lagrange interpolation (lsq_degree 0),
 * uniform tree (leaf_max 0), spectrum chunks chosen at tree build (freq_chunks 0). */
void dfmm_default_params(dfmm_params* p);

/* Precompute a plan (Sec. 4.1, Eq. m2l and Theorem 1): for every level 2..D
 * the kernel on the lattice of node offsets, the block-Toeplitz generators
 * of the stored offsets (158, or 16 with DFMM_M2L_FFT_SYM) and their DFTs;
 * with DFMM_KERNEL_SURROGATE (cubic media) the network is trained first.
 * The operators depend only on the kernel, not on the segments, and are
 * reused by every tree and every call.  Synchronous.
 * Errors: DFMM_E_ARG for out-of-range parameters or a stiffness that is not
 * positive definite; DFMM_E_NOMEM; DFMM_E_HIP. */
int dfmm_fmm_setup(const dfmm_params* prm, void* stream, dfmm_plan** out);

/* Build the octree of the quadrature points of seg (device, [n_seg][2][3]):
 * Morton keys, a stable radix sort, occupied cells per level, 27-neighbour
 * lists of the leaves and interaction lists (children of the parent's
 * neighbours that are not neighbours; Sec. 4.3) on levels 2..D, and every
 * workspace dfmm_fmm_forces needs.  Synchronises the stream.  n_seg >= 1.
 * With DFMM_MIXED a level may hold at most 2^23 - 1 occupied cells (the M2L
 * list entries are 32-bit words).
 * Errors: DFMM_E_NONFINITE / DFMM_E_OUT_OF_BOX for bad coordinates,
 * DFMM_E_ARG (also for the cell limit), DFMM_E_NOMEM, DFMM_E_HIP. */
int dfmm_build_tree(dfmm_plan* plan, const double* seg, int64_t n_seg, void* stream,
                    dfmm_tree** out);

/* Forces on all n_seg segments (forces: device [n_seg][2][3]) by the
 * Lagrange FMM of Alg. lagrange.  seg must hold the same positions the tree
 * was built from; burgers is device [n_seg][3].  Asynchronous on `stream`;
 * allocates nothing.  Errors: DFMM_E_ARG, DFMM_E_STATE (tree from another
 * plan), DFMM_E_HIP. */
int dfmm_fmm_forces(const dfmm_plan* plan, dfmm_tree* tree, const double* seg,
                    const double* burgers, double* forces, void* stream);

/* Debug check for the condition dfmm_fmm_forces relies on: seg (device,
 * [n_seg][2][3], the tree's n_seg) holds the positions the tree was built
 * from.  Every quadrature point is formed again as the force call forms it
 * (Sec. 2: x1 + (1 + u_k)/2 dS) and compared bit for bit with the copy the
 * build kept.  Synchronises the stream.  Errors: DFMM_E_STATE if any point
 * differs (the message gives the count and the first segment) or the tree is
 * from another plan; DFMM_E_ARG, DFMM_E_HIP. */
int dfmm_tree_check_positions(const dfmm_plan* plan, dfmm_tree* tree, const double* seg, void* stream);

/* Direct O(N^2) forces on the target segments targets[0..n_targets)
 * (device int64 indices into seg; NULL = all segments, then n_targets must
 * equal n_seg) from every quadrature point of every segment, Eq. stress3.
 * forces: device [n_targets][2][3].  fp32 = 1 evaluates pairs in float with
 * compensated float accumulation; 0 in double.  Asynchronous.
 * Errors: DFMM_E_ARG, DFMM_E_HIP. */
int dfmm_direct_forces(const dfmm_plan* plan, const double* seg, const double* burgers,
                       int64_t n_seg, const int64_t* targets, int64_t n_targets,
                       double* forces, int fp32, void* stream);

/* dfmm_direct_forces without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same sum, arguments and results as dfmm_direct_forces;
 * its scratch (sorted points, per-chunk partial stresses, per-point stress)
 * lives in a fixed array of DFMM_NOALLOC_SCRATCH_BYTES in the library, one
 * copy per GPU, held until the process ends.  Calls that overlap on one GPU
 * (other streams, other threads) race on that array and must not be made.
 * With targets != NULL the indices are checked first, which synchronises
 * the stream; otherwise the call is asynchronous.  Errors: DFMM_E_ARG (also
 * when the sizes need more scratch than the array holds: about 72 bytes per
 * quadrature point plus 48 per target point and source chunk; 60,000
 * segments with all of them as targets fit), DFMM_E_HIP. */
#define DFMM_NOALLOC_SCRATCH_BYTES (64ll << 20)
int dfmm_direct_forces_noalloc(const dfmm_plan* plan, const double* seg, const double* burgers,
                               int64_t n_seg, const int64_t* targets, int64_t n_targets,
                               double* forces, int fp32, void* stream);
/* Scratch bytes dfmm_direct_forces_noalloc needs for these sizes (0 on bad
 * arguments). */
size_t dfmm_direct_noalloc_bytes(const dfmm_plan* plan, int64_t n_seg, int64_t n_targets);

/* Per-stage timing of dfmm_fmm_forces with HIP events on its stream.
 * on = 1 starts recording (resetting the accumulators), 0 stops.  While
 * on, every dfmm_fmm_forces call records events around each stage.
 * dfmm_tree_stage_times synchronises the tree's last stream and writes the
 * accumulated milliseconds per stage and the number of timed calls:
 * ms[0..DFMM_N_STAGES).  Stages: 0 points+P2M, 1 M2M, 2 forward DFT,
 * 3 M2L Hadamard product, 4 inverse DFT, 5 L2L, 6 near field+L2P,
 * 7 force assembly. */
#define DFMM_N_STAGES 8
int dfmm_tree_set_timing(dfmm_tree* tree, int on);
int dfmm_tree_stage_times(dfmm_tree* tree, double* ms, int* n_calls);

/* ---------------------------------------------------------------------
 * Learned surrogate for the anisotropic Green's-function derivative (the
 * costly kernel evaluation of Sec. 2, done numerically for anisotropic
 * media).  A network 6 -> 4 x hidden (SiLU) -> 18 maps the unit direction and
 * the normalised (c11, c12, c44) to the 18 distinct components of
 * c44 (Phi - Phi_iso[Voigt]) / scale, Phi_vpq = r^2 d_q G_vp (singular part).
 * It is trained on the GPU by the library's own forward, backward and Adam
 * kernels on directions drawn from a counter-based generator, with targets
 * from the library's double-precision circle quadrature.  A cube map of
 * direction bins (6 x bins x bins) records the network's largest error per
 * bin on validation directions, relative to the largest component of Phi;
 * bins above `tol` keep the exact quadrature. */
typedef struct {
  int hidden;          /* hidden width; 128                                   */
  int epochs;          /* passes over the training samples                     */
  int batch;           /* rows per optimisation step                           */
  int bins;            /* cube-map bins per face edge (1..256)                 */
  int64_t n_samples;   /* training directions                                  */
  double lr;           /* Adam step size, cosine-decayed to 1% of it           */
  double tol;          /* residual gate (1e-5)                                 */
  uint64_t seed;       /* generator seed                                       */
} dfmm_surrogate_cfg;

/* Defaults: hidden 128, 2,000,000 samples, 20 epochs, batch 4096, lr 1e-3,
 * tol 1e-5, 32 bins, seed 1. */
void dfmm_surrogate_default_cfg(dfmm_surrogate_cfg* cfg);

/* Train the surrogate of an anisotropic plan and build its residual gate.
 * Every product of the forward and backward passes runs on the matrix cores
 * (f16 operands, f32 accumulation, f32 master weights and Adam moments).
 * Synchronous.  A surrogate in use is switched off first (and the operator
 * spectra rebuilt with the exact kernel); the new one is not switched on
 * (see dfmm_surrogate_use).  Not to be called while other calls use the
 * plan.  DFMM_E_ARG for an isotropic plan or a bad configuration. */
int dfmm_surrogate_train(dfmm_plan* plan, const dfmm_surrogate_cfg* cfg, void* stream);

/* on = 1: rebuild the plan's M2L spectra with the surrogate where its bin
 * passes the gate (exact quadrature elsewhere) and use it in the near field
 * of the float path; on = 0: back to the exact kernel everywhere (spectra
 * rebuilt exactly as dfmm_fmm_setup built them).  The network is evaluated
 * on the matrix cores (f16 weights and activations, f32 accumulation), the
 * same arithmetic the gate judged.  Synchronous; trees built with the plan
 * stay valid. */
int dfmm_surrogate_use(dfmm_plan* plan, int on, void* stream);

/* JSON: training loss per epoch, fraction of gated-in bins, max / median bin
 * error, training time. */
int dfmm_surrogate_info(const dfmm_plan* plan, char* json, size_t cap);

/* Network parameters as float32 in layer order (W row-major [out][in], then
 * b), host memory.  get: *n receives the count, copied if cap >= count.
 * set: allocates the network if needed, switches a surrogate in use off
 * (spectra rebuilt exactly) and leaves the network untrained (no gate; it
 * cannot be switched on).  For testing. */
int dfmm_surrogate_get_params(const dfmm_plan* plan, float* host, int64_t cap, int64_t* n);
int dfmm_surrogate_set_params(dfmm_plan* plan, const float* host, int64_t n);

/* The residual gate: mask[(face * bins + i) * bins + j] = 1 where the
 * network is used (face = 2 axis + (T_axis < 0), (i, j) the cube-map cell of
 * the other two coordinates over |T_axis|, in axis order after the face's
 * axis, cyclically), host memory; *bins receives the bins per face edge and
 * the mask is copied if cap >= 6 bins^2.  DFMM_E_STATE without a gate. */
int dfmm_surrogate_get_gate(const dfmm_plan* plan, unsigned char* mask, int64_t cap, int* bins);

/* Persistence of a trained surrogate (network, gate, its statistics) in a
 * binary file of this library.  save: DFMM_E_STATE without a trained
 * network, DFMM_E_ARG if the file cannot be written.  load: DFMM_E_ARG for
 * an isotropic plan or a file that is not one of these, DFMM_E_STATE if the
 * network was trained for another medium; switches a surrogate in use off
 * (spectra rebuilt exactly); the loaded one is trained but not switched on.
 * Synchronous. */
int dfmm_surrogate_save(const dfmm_plan* plan, const char* path);
int dfmm_surrogate_load(dfmm_plan* plan, const char* path, void* stream);

/* Mean-squared loss over rows x 18 outputs and its gradient (device float
 * [n_params]) for device rows X [n][6], Y [n][18], by the training path; and
 * the network output Y = net(X) by the inference path the kernels use.
 * Synchronous.  For gradient checks. */
int dfmm_surrogate_loss_grad(dfmm_plan* plan, const float* X, const float* Y, int64_t n, float* grad,
                             double* loss, void* stream);
int dfmm_surrogate_forward(const dfmm_plan* plan, const float* X, int64_t n, float* Y, void* stream);

/* ---------------------------------------------------------------------
 * Many independent configurations in one launch.  dfmm_batch_create
 * captures, into one HIP graph, the dfmm_fmm_forces launches of n_cfg
 * (plan, tree, seg, burgers, forces) tuples spread over n_lanes parallel
 * branches (configurations assigned longest-first to the least loaded
 * branch, by estimated cost), plus a timestamp kernel after each
 * configuration.  The device arrays are bound at creation and must stay
 * valid; trees must not be rebuilt while the batch exists.  dfmm_batch_run
 * launches the graph on `stream` (asynchronous).  dfmm_batch_latencies
 * synchronises and returns, per configuration, the milliseconds from the
 * start of the last run to the retirement of that configuration's last
 * kernel (device wall clock).  Errors: DFMM_E_ARG, DFMM_E_STATE (a tree
 * timing switch is on), DFMM_E_HIP. */
typedef struct dfmm_batch dfmm_batch;
int dfmm_batch_create(const dfmm_plan* const* plans, dfmm_tree* const* trees, const double* const* seg,
                      const double* const* burgers, double* const* forces, int n_cfg, int n_lanes,
                      void* stream, dfmm_batch** out);
int dfmm_batch_run(dfmm_batch* batch, void* stream);
/* One-shot form: the n_cfg force evaluations in one graph launch over
 * min(4, n_cfg) branches (dfmm_batch_create, run, destroy), for callers that
 * evaluate a set of configurations once.  Same arguments and errors as
 * dfmm_batch_create; synchronous (returns when every forces[i] is written);
 * allocates the graph and its streams for the duration of the call. */
int dfmm_forces_batched(const dfmm_plan* const* plans, dfmm_tree* const* trees, const double* const* seg,
                        const double* const* burgers, double* const* forces, int n_cfg, void* stream);
/* Launch-shape autotuner of the batch graph: the same n_cfg evaluations
 * captured with 1, 2, 4 and 8 parallel branches (counts above n_cfg are
 * skipped, 1 always tried), each graph replayed `reps` times after one
 * warm-up; *best = the branch count with the smallest mean time per replay
 * (ms[0..3], if non-NULL: that mean for 1, 2, 4, 8 branches, 0 where not
 * tried).  The forces are written by every replay.  Synchronous; allocates
 * (one graph at a time).  Errors: as dfmm_batch_create, DFMM_E_ARG for
 * reps < 1. */
int dfmm_autotune_batch_lanes(const dfmm_plan* const* plans, dfmm_tree* const* trees, const double* const* seg,
                              const double* const* burgers, double* const* forces, int n_cfg, int reps, void* stream,
                              int* best, double* ms);
int dfmm_batch_latencies(dfmm_batch* batch, double* ms, int n_cfg);
void dfmm_batch_destroy(dfmm_batch* batch);

/* Depth autotuner (App. B: near-field cost ~ C_n x near pairs, far-field
 * cost ~ C_f x M2L translations; the optimum balances them).  Builds the
 * tree of seg at each depth in [d_min, d_max], times one dfmm_fmm_forces at
 * the plan's depth (prm->depth, which must lie in the range) to measure C_n,
 * C_f and the per-cell cost of the other stages, and predicts every
 * candidate's time from its exact pair counts (pred_ms[d - d_min] if
 * non-NULL).  The model's fastest depth and its two neighbours are then
 * set up and timed, and the fastest measured one is returned in *best
 * (measured ms per depth in meas_ms[d - d_min] if non-NULL; 0 where not
 * measured).  Synchronous; allocates.  seg/burgers: device. */
int dfmm_autotune_depth(const dfmm_params* prm, const double* seg, const double* burgers, int64_t n_seg,
                        int d_min, int d_max, void* stream, int* best, double* pred_ms, double* meas_ms);

/* JSON descriptions: parameters, M2L operator memory (Eq. mem_unif and the
 * stored spectra), precompute time / tree sizes per level, pair counts, and
 * for a tree whether its near field takes one kernel evaluation per
 * unordered pair ("symmetric_near": cubic media, uniform tree, leaves of at
 * most 1024 points) or one per ordered pair. */
int dfmm_plan_info(const dfmm_plan* plan, char* json, size_t cap);
int dfmm_tree_info(const dfmm_tree* tree, char* json, size_t cap);

/* NULL-safe destructors. */
void dfmm_tree_destroy(dfmm_tree* tree);
void dfmm_plan_destroy(dfmm_plan* plan);

const char* dfmm_status_string(int status);
const char* dfmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFMM_H */
