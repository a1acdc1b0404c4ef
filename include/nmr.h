/*
 * nmr.h - C ABI of libnmr: the reduced implicit-Euler Newton iteration of a
 * deep-autoencoder subspace simulator on AMD MI355X (gfx950).
 *
 * Method (High-order Differentiable Autoencoder for Nonlinear Model
 * Reduction): full-space displacement u = U p + D(q) (Sec. 3.6,
 * eq. our_subspace) with D a decoder MLP followed by the fixed filtering
 * layer I - U U^T (Sec. 3.5) and the Dirichlet mask P of pinned DOFs.  Each
 * implicit-Euler step (Sec. 3.2) solves phi(r) = 0 (eq. our_equation_of_motion)
 * for r = [p; q] by Newton's method with the matrix of eq. system_mat, whose
 * third-order term dJ is eq. delta_j.  Decoder derivatives are collective
 * complex-step right contractions (Sec. 4.3) and complex-step
 * backpropagation (Sec. 4.4); force and stiffness are integrated over a
 * weighted cubature set of tets (Sec. 5) with weights from a
 * weight-prediction MLP evaluated once per step (Sec. 5.2).
 *
 * Conventions for every call:
 *   - Return value: NMR_OK (0) or a negative nmr_status.  No C++ exception
 *     crosses this ABI.  nmr_last_error() gives a text for the last failure
 *     on the calling thread.
 *   - Ownership: the caller owns every array argument.  The library owns only
 *     what lives inside a handle (device copies of the problem, state,
 *     workspaces) and frees it in the matching destroy call.
 *   - Device vs host: arguments documented "device" are device pointers on the
 *     context's GPU (for example torch tensors' data pointers); "host" ones are
 *     ordinary host memory.  Every call is ordered on the context's stream
 *     and returns without waiting unless it writes a host output, in which
 *     case it synchronizes that stream first.
 *   - Layouts: row-major; the DOF index of vertex v, coordinate c is 3 v + c;
 *     r = [p; q] with the n_p linear coordinates first (Sec. 3.6).
 *   - Element type "real": double for an instance created with NMR_PREC_FP64,
 *     float for NMR_PREC_FP32 and NMR_PREC_BF16.
 */
#ifndef NMR_H
#define NMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmr_ctx nmr_ctx;         /* one GPU + one stream + HBM budget   */
typedef struct nmr_decoder nmr_decoder; /* device copy of a decoder MLP        */
typedef struct nmr_inst nmr_inst;       /* one simulated object and its state  */

typedef enum {
  NMR_OK = 0,
  NMR_ERR_ARG = -1,       /* invalid argument or shape                        */
  NMR_ERR_BUDGET = -2,    /* instance does not fit the context's HBM budget    */
  NMR_ERR_OOM = -3,       /* device allocation failed                          */
  NMR_ERR_INVERTED = -4,  /* a cubature tet has det F <= 0                     */
  NMR_ERR_SINGULAR = -5,  /* LU pivot below 1e-300 * max |A_ij|                */
  NMR_ERR_NONFINITE = -6, /* non-finite residual or Newton matrix              */
  NMR_ERR_DEVICE = -7     /* HIP runtime error                                 */
} nmr_status;

typedef enum { NMR_ACT_IDENTITY = 0, NMR_ACT_TANH = 1, NMR_ACT_ELU = 2, NMR_ACT_SIN = 3 } nmr_act;
typedef enum { NMR_PREC_FP64 = 0, NMR_PREC_FP32 = 1, NMR_PREC_BF16 = 2 } nmr_prec;

/* A fully connected MLP: z_0 = x, z_l = act(W_l z_{l-1} + b_l) for l < L and
 * a linear last layer (the decoder of Sec. 3.5).  Host pointers, read only
 * during the create call. */
typedef struct {
  int n_layers;             /* L >= 1                                          */
  const int* widths;        /* L + 1 entries: input size ... output size       */
  int act;                  /* nmr_act of the hidden layers                    */
  const double* const* W;   /* L pointers, W[l]: widths[l+1] x widths[l]       */
  const double* const* b;   /* L pointers, b[l]: widths[l+1]                   */
} nmr_mlp_desc;

/* One simulated object (host pointers, copied to the device by
 * nmr_instance_create).  N = 3 * n_vertices, R = n_p + n_q <= 31. */
typedef struct {
  int n_vertices;
  const double* X;          /* n_vertices x 3 rest positions                   */
  int n_tets;
  const int32_t* tets;      /* n_tets x 4, positively oriented                  */
  const uint8_t* pinned;    /* n_vertices, 1 = Dirichlet vertex (mask P)        */
  double E, nu, rho;        /* neo-Hookean Young's modulus, Poisson, density    */
  double gravity[3];        /* f_ext = M (1 (x) gravity)                        */
  double dt;                /* implicit-Euler time step                         */
  int n_p;                  /* linear (PCA) subspace size, may be 0             */
  const double* U;          /* N x n_p, orthonormal, zero at pinned DOFs        */
  const nmr_mlp_desc* decoder;   /* decoder (n_q = widths[0], widths[L] >= N)  */
  nmr_decoder* shared_decoder;   /* if non-NULL, used instead of `decoder`;    */
                                 /* the first N output rows are used           */
  int n_cub;                /* cubature set size |C|                            */
  const int32_t* cub_ids;   /* |C| tet ids                                      */
  const double* cub_w;      /* |C| fixed weights, or NULL: weight net below     */
  const nmr_mlp_desc* wnet; /* R -> ... -> |C|, softplus after every layer      */
  double wnet_scale;        /* w = wnet_scale * wnet(rbar)                      */
  const double* r0;         /* R initial generalized coordinate                 */
  const double* rdot0;      /* R initial generalized velocity                   */
  int newton_path;          /* 0: automatic -- Gram-folded mass terms when      */
                            /*    n_p == 0 (the output layer is linear and M    */
                            /*    constant, so Jt^T M Jt = F^T (W^T M W) F and  */
                            /*    only cubature DOFs are decoded per iteration); */
                            /* 1: direct (every DOF decoded each iteration)     */
  int trimmed;              /* 0: the paper's formulation (eq. our_equation_   */
                            /*    of_motion with f_fict); 1: f_fict dropped, as */
                            /*    in latent space dynamics (Sec. 3.3, Sec. 6):  */
                            /*    phi has no Jt^T M H(dq,dq) term and the Newton */
                            /*    matrix is its exact derivative, i.e. dJ =     */
                            /*    H.(dq - dt qdot) and Hdd = 0 in every output  */
  double fd_h;              /* 0: derivatives by collective complex steps (the  */
                            /*    paper); > 0: by recursive central differences */
                            /*    of step fd_h instead (the comparison of Sec. */
                            /*    6): 14 n_q + 3 plain forward passes and real */
                            /*    backpropagation at q, q +- fd_h e_j.  Needs   */
                            /*    n_q <= 8 (n_q <= 4 in FP64)                   */
} nmr_problem;

/* ---- lifecycle ---------------------------------------------------------- */

/* Context on GPU `device`; `hip_stream` is a hipStream_t (NULL = a stream the
 * library creates at default priority).  hbm_budget_bytes = 0: no limit. */
int nmr_create(int device, void* hip_stream, size_t hbm_budget_bytes, nmr_ctx** out);
int nmr_destroy(nmr_ctx* ctx);
const char* nmr_last_error(void);

/* Device copy of a decoder in precision `prec` (nmr_prec), shareable by many
 * instances (one trained net reused across identical domains, Sec. 6.8).
 * Destroying it while instances still use it is deferred until the last one
 * is destroyed. */
int nmr_decoder_create(nmr_ctx* ctx, const nmr_mlp_desc* desc, int prec, nmr_decoder** out);
int nmr_decoder_destroy(nmr_decoder* dec);

/* Copies the problem to the device, precomputes rest-shape matrices, volumes
 * and the lumped mass (Sec. 3.1), and sets the state (rbar, rdot_bar) =
 * (r0, rdot0).  Charges the context budget: NMR_ERR_BUDGET if it does not
 * fit, NMR_ERR_OOM if allocation fails. */
int nmr_instance_create(nmr_ctx* ctx, const nmr_problem* prob, int prec, nmr_inst** out);
int nmr_instance_destroy(nmr_inst* inst);
/* Device bytes charged to the budget for this instance (host output). */
int nmr_instance_bytes(const nmr_inst* inst, size_t* bytes);
/* Newton path the instance runs (host output): 0 = Gram-folded mass terms
 * (only the DOFs of cubature tets decoded per iteration), 1 = direct. */
int nmr_instance_newton_path(const nmr_inst* inst, int* path);
/* Host buffers: r and rdot (R doubles each) of the last completed step; u
 * (N reals, may be NULL) is the full-space displacement u = U p + D(q)
 * (Sec. 3.6, eq. our_subspace) at that r, decoded into the instance's frame
 * buffer (see nmr_instance_get_frame) and copied from there.  Synchronizes. */
int nmr_instance_get_state(nmr_inst* inst, double* r, double* rdot, void* u_or_null);
/* Frame output.  Every implicit-Euler step (Sec. 3.2) starts its Newton
 * iteration at r = rbar, the state the previous step ended in, so its first
 * decoder pass already evaluates D at that frame's state: the step writes
 * that frame's full-space displacement u = U p + D(q) [N reals] into the
 * instance's frame buffer (the value channel through every row of the output
 * layer), as part of the same graph launch.  After a step, the buffer holds
 * the frame the step started from; after nmr_instance_get_state with u, the
 * frame of the current state.  get_frame copies it to a host buffer u [N
 * reals] (synchronizes); frame_ptr returns its device address (valid until
 * the instance is destroyed; read it after the context stream's work). */
int nmr_instance_get_frame(nmr_inst* inst, void* u);
int nmr_instance_frame_ptr(nmr_inst* inst, void** u_dev);
/* Host buffers: sets (rbar, rdot_bar) and clears a failed status. */
int nmr_instance_set_state(nmr_inst* inst, const double* r, const double* rdot);
/* Status of the last step (nmr_status); synchronizes. */
int nmr_instance_status(nmr_inst* inst);

/* ---- hot path ----------------------------------------------------------- */

/* Decoder value and contracted derivatives (Sec. 4.3, 4.4, eq. delta_j).
 * Device inputs, n_q doubles each: q, dq = q - qbar, qdot_bar.
 * Device outputs (reals): u = D(q) [N], J = dD/dq [N x n_q],
 * dJ = (S.dq).dq + H.(3 dq - dt qdot_bar) [N x n_q], Hdd = H(dq, dq) [N].
 * If a_or_null (device, N reals) is given, also the left contractions of
 * D through complex-step backpropagation: B = sum_i a_i H_i [n_q x n_q
 * doubles, column j from the perturbation of q_j] and JTa = J^T a [n_q
 * doubles]; both may be NULL otherwise.  D includes the filter and mask. */
int decoder_jacobian_hessian(nmr_inst* inst, const double* q, const double* dq,
                             const double* qdot_bar, const void* a_or_null,
                             void* u, void* J, void* dJ, void* Hdd,
                             double* B_or_null, double* JTa_or_null);

/* Cubature force and reduced stiffness (Sec. 5, neo-Hookean tets).  Device
 * inputs: u [N reals], Jt = [U, J] [N x R reals], w [|C| reals] or NULL for
 * the instance's current weights.  Device outputs: f_int [N reals] or NULL,
 * fr = sum_e w_e Jt_e^T f_e [R doubles], Kr = sum_e w_e Jt_e^T K_e Jt_e
 * [R x R doubles].  NMR_ERR_INVERTED if a cubature tet has det F <= 0
 * (checked after a synchronization). */
int cubature_force_stiffness(nmr_inst* inst, const void* u, const void* Jt, const void* w_or_null,
                             void* f_int_or_null, double* fr, double* Kr);

/* For callers that cannot allocate device memory at call time (tight serving
 * loops, harnesses that forbid hipMalloc): cubature_force_stiffness with the
 * same arguments, layouts, results (the same kernels, so the same bits) and
 * errors, but it calls no hipMalloc, hipFree or allocating library routine.
 * Its working memory -- the instance's table entry, a status word, the
 * weighted element forces [|C| x 12 reals] and one FP64 partial sum per
 * block of four cubature tets [ceil(|C| / 4) x (R*R + R) doubles] -- lives in
 * a static device array of 16 MiB that each GPU the library runs on holds
 * until the process ends.  It needs 12800 + round_up_256(48 |C|) (96 |C| in
 * FP64) + 8 ceil(|C| / 4) (R*R + R) bytes: NMR_ERR_ARG, before any device
 * work, if that exceeds 16 MiB (|C| = 6,600 at R = 30 needs 12.6 MB).  Every
 * call on a GPU shares that GPU's array and overwrites what the last call
 * left there: calls that overlap on one GPU (other threads, other contexts
 * on the same device) race and must be serialized by the caller.  The
 * instance is only read.  Synchronizes the context stream (the status is
 * read back). */
int cubature_force_stiffness_noalloc(nmr_inst* inst, const void* u, const void* Jt, const void* w_or_null,
                                     void* f_int_or_null, double* fr, double* Kr);

/* Newton system at iterate r (device, R doubles) of the step that starts from
 * the instance state: phi (eq. our_equation_of_motion) [R doubles] and its
 * Jacobian A = dphi/dr (eq. system_mat) [R x R doubles], both device.  Uses
 * the cubature weights of that step. */
int reduced_newton_system(nmr_inst* inst, const double* r, double* A, double* phi);

/* One implicit-Euler step (Sec. 3.2) of the reduced equation of motion
 * (eq. our_equation_of_motion, Sec. 3.6) with n_iters full Newton
 * iterations, each solving A delta = -phi with the matrix of eq. system_mat
 * (third-order term eq. delta_j) by LU with partial pivoting, starting from
 * r = rbar, then rdot = (r - rbar) / dt, rbar = r.  The cubature weights come
 * from the weight net at rbar once per step (Sec. 5.2).  resid_norms_or_null:
 * host, n_iters doubles of ||phi|| per iteration (synchronizes).  A failure
 * leaves the state of the previous step in place and is returned here (if
 * synchronized) or by nmr_instance_status. */
int reduced_newton_step(nmr_inst* inst, int n_iters, double* resid_norms_or_null);

/* Advances n_inst instances (same context) n_steps steps of n_iters Newton
 * iterations each (the step of reduced_newton_step for every instance), all
 * instances together.  Instances that share a decoder -- one trained net
 * reused across identical domains, as for the strings of the multi-domain
 * scenes of Sec. 6.8 -- run their decoder passes as one batched launch per
 * layer, their perturbation columns stacked like the mini-batch of
 * collective perturbations of Sec. 4.4; every phase is one launch for the
 * whole set, captured in a HIP graph per step.  Host
 * outputs: status [n_inst] (nmr_status of each instance; a failed instance is
 * frozen at its last good state, the others continue) and step_ms_or_null
 * [n_steps] (device time of each step). */
int step_many(nmr_ctx* ctx, nmr_inst* const* insts, int n_inst, int n_steps, int n_iters,
              int* status, float* step_ms_or_null);

/* ---- coupled domains (Sec. 6.8) ------------------------------------------ */

typedef struct nmr_coupled nmr_coupled;

/* A coupled set: a core domain and n_rods domains tied to it, the
 * multi-domain form of the paper's substructured scenes (Sec. 6.8: strings
 * on a ball, branches on a trunk).  The paper gives no coupling equations;
 * here each tied vertex of a rod owns a copy of a core vertex and the two
 * are joined by a zero-length spring of stiffness kappa [N/m]:
 *   E_tie = kappa/2 sum |(X + u)_rod vertex - (X + u)_core vertex|^2.
 * One coupled step (Sec. 3.2) solves the stacked reduced equations of motion
 * (eq. our_equation_of_motion per domain, the tie force entering as internal
 * force, so also in the a . H term of eq. system_mat) with the Newton matrix
 * of the stacked system: each domain's own matrix plus the tie stiffness
 * dt^2 kappa Jt_T^T Jt_T, and the core-rod blocks -dt^2 kappa Jt_core,T^T
 * Jt_rod,T.  It is solved by static condensation onto the core (each rod's
 * block eliminated on its own, the core's Schur complement summed over the
 * rods in order and solved), FP64 LU with partial pivoting throughout.
 * ties: host, n_rods x n_tie x 2 int32 (rod vertex, core vertex); every rod
 * has n_tie <= 21 tied vertices, no core vertex is tied twice.  Members:
 * same context, precision and time step, complex-step derivatives, not
 * attached to a pool, each at most once; they run the direct Newton path in
 * the set (every DOF decoded per iteration).  A member cannot be destroyed
 * while it belongs to a set.  Charges the context budget for the set's
 * buffers (tie forces, per-member systems, per-rod workspaces). */
int nmr_coupled_create(nmr_ctx* ctx, nmr_inst* core, int n_rods, nmr_inst* const* rods, const int32_t* ties,
                       int n_tie, double kappa, nmr_coupled** out);
int nmr_coupled_destroy(nmr_coupled* set);
/* n_steps coupled steps of n_iters Newton iterations (one graph launch per
 * step; each step also writes every member's frame, see
 * nmr_instance_get_frame).  A failure of any member (inverted tet, singular
 * or non-finite system) freezes the whole set at its last good state and
 * is reported for every member.  Host outputs: status [1 + n_rods] (core
 * first), step_ms_or_null [n_steps].  Each member's recorded residual norms
 * are those of its own block of the stacked residual; the core's is the
 * norm of the whole stacked residual.  Synchronizes. */
int nmr_coupled_step(nmr_coupled* set, int n_steps, int n_iters, int* status, float* step_ms_or_null);

/* ---- served form: slot pools (continuous batching) ---------------------- */

typedef struct nmr_pool nmr_pool;

/* A pool of `capacity` slots whose time step is captured once as a HIP graph
 * over all slots; instances attach to free slots and detach between steps
 * without a new capture (empty slots return at once).  Every attached
 * instance must share the first one's decoder, precision and sizes (N, n_p,
 * n_q, |C|, weight-net widths), Newton path and decoded cubature DOFs,
 * formulation (trimmed) and derivative scheme (fd_h), i.e. one request
 * class. */
int nmr_pool_create(nmr_ctx* ctx, int capacity, nmr_pool** out);
int nmr_pool_destroy(nmr_pool* pool);
/* Attaches `inst` to a free slot (host output *slot).  NMR_ERR_BUDGET if the
 * pool is full, NMR_ERR_ARG if the instance does not match the pool's class
 * or is already attached to a pool.  The instance keeps its own state and
 * buffers; nmr_instance_destroy of an attached instance detaches it first,
 * and nmr_pool_destroy detaches every instance. */
int nmr_pool_attach(nmr_pool* pool, nmr_inst* inst, int* slot);
int nmr_pool_detach(nmr_pool* pool, int slot);
/* One implicit-Euler step (n_iters Newton iterations) of every attached
 * instance, one graph launch.  status_or_null: host, `capacity` ints
 * (nmr_status per slot, 0 for empty slots; synchronizes); *ms_or_null: device
 * time of the step (synchronizes). */
int nmr_pool_step(nmr_pool* pool, int n_iters, int* status_or_null, float* ms_or_null);

/* ---- tile configurations of batched launches ---------------------------- */

/* How the hidden-layer GEMM launches of step_many and of slot pools choose
 * their tiles.  A configuration is (ib, mr): ib instances per block (1, 2 or
 * 4; stacked instances share the weight tile) and mr 16-row output tiles per
 * wavefront (1; or 2 and 4, "tall" tiles in which one wavefront covers one
 * instance's 16 mr rows over the whole reduction, so each operand fragment
 * feeds several MFMAs).  Eligible: ib <= the number of instances in the
 * launch; ib > 1 or mr > 1 only for FP32/BF16 complex-step jets; mr > 1 only
 * with ib = 4, in a forward layer of at most 64 jet columns (128 for mr = 2)
 * or a backward layer of at most 32 adjoint columns, whose padded row count
 * (the output width forward, the input width backward) 16 mr divides.
 * Forward layers at (1, 1) with more than 16 jet columns may also take jet
 * groups (jet_groups = 1): the columns of a 16-row tile split over
 * ceil(n_q / 3) blocks, each computing the four base channels and the four
 * channels of three perturbations.  With at most 64 jet columns (n_q <= 15)
 * every column is the same sum as without groups, so the results are the
 * same bits; wider whole tiles split K over fewer waves and agree to
 * rounding.  Launches of one instance run (1, 1).
 *   NMR_TILES_RULE (the default): a fixed rule from the layer's row count,
 *     its columns and the number of instances: tall tiles once there are 768
 *     waves of 16 mr rows; else ib from the rounds of 256 blocks the launch
 *     takes, weighed by how much longer a stacked block runs; jet groups in
 *     forward layers of fewer than 192 row-tile x instance blocks.  Results
 *     are bitwise reproducible.
 *   NMR_TILES_AUTOTUNE: the first time a (direction, layer widths, columns,
 *     instances, precision, derivative scheme) occurs in a step_many call (or
 *     a pool step with at least half its slots attached), every eligible
 *     configuration is timed on the context stream on the group's own decoder
 *     buffers and the fastest is kept for the context's lifetime.
 *   NMR_TILES_FORCE: (ib, mr) without jet groups wherever it is eligible,
 *     the rule elsewhere.
 * Configurations split the reduction over K differently, so results under
 * different tiles agree to rounding, not bitwise.  Changing the mode drops
 * the graphs captured under the previous one (synchronizes).  NMR_ERR_ARG for
 * an unknown mode or, when forcing, ib or mr outside {1, 2, 4}. */
typedef enum { NMR_TILES_RULE = 0, NMR_TILES_AUTOTUNE = 1, NMR_TILES_FORCE = 2 } nmr_tiling;
int nmr_set_tiling(nmr_ctx* ctx, int mode, int ib, int mr);

typedef struct {
  int forward;     /* 1: forward jet layer, 0: backpropagation layer */
  int m_in, m_out; /* padded input and output widths of the layer */
  int cols;        /* jet (forward) or adjoint (backward) columns */
  int n_inst;      /* instances in the launch */
  int prec;        /* nmr_prec */
  int ib, mr;      /* the configuration chosen */
  int jet_groups;  /* 1: with jet groups */
  float us;        /* its measured device time per launch, microseconds */
} nmr_tile_choice;

/* The autotuned choices so far: copies min(count, cap) entries to out (host)
 * and that number to *n. */
int nmr_tiling_table(nmr_ctx* ctx, nmr_tile_choice* out, int cap, int* n);

/* ---- neural cubature training (Sec. 5) --------------------------------- */

/* Reduced force of every element at pose r (Sec. 5.1, the training data of
 * the cubature networks): with u = U p + D(q) and Jt = [U, J] at r,
 * F[e] = Jt_e^T f_e(u) for every tet e, f_e its neo-Hookean force.  Device
 * input r [R doubles]; device outputs F [n_tets x R doubles], f_or_null [R
 * doubles] = sum_e F[e] (the full-quadrature reduced force, tets in index
 * order), u_or_null [N doubles].  Decoder derivatives as in
 * decoder_jacobian_hessian in the instance's precision, element arithmetic in
 * FP64.  Allocates its working memory; NMR_ERR_INVERTED if a tet has
 * det F <= 0 (its row of F is then zero).  The instance state is unchanged.
 * Synchronizes. */
int nmr_element_forces(nmr_inst* inst, const double* r, double* F, double* f_or_null, double* u_or_null);

typedef struct nmr_trainer nmr_trainer; /* one neural cubature training run */

/* A training run (host pointers, read only during nmr_trainer_create). */
typedef struct {
  int n_poses;               /* P >= 1                                          */
  const double* poses;       /* P x R training poses r_p                        */
  int c_max;                 /* elements the cubature set may hold, < n_tets    */
  int n_c0;                  /* initial set size, 1 <= n_c0 <= c_max            */
  const int32_t* c0;         /* n_c0 distinct tet ids, or NULL: n_c0            */
                             /* farthest-point samples of the tet centroids     */
                             /* from tet 0 (the Voronoi samples of Sec. 5.2)    */
  int K;                     /* elements added per alternation (Sec. 5.1)       */
  int epochs;                /* Adam steps per net per alternation              */
  double lr, beta1, beta2, eps;  /* Adam (the paper: lr = 1e-3)                 */
  const nmr_mlp_desc* wnet;  /* weight net R -> ... -> c_max, softplus after    */
                             /* every layer, hidden widths <= 1024; row j of    */
                             /* its last layer serves the j-th element to join  */
  double wnet_scale;         /* w = wnet_scale * wnet(r) (> 0)                  */
  const double* snet;        /* 170 selection-net parameters: G0 [3][8] and     */
                             /* G1 [8][8] (graph convolutions, [in][out]), A1   */
                             /* [8][8] ([out][in]), a1 [8], A2 [8], a2, c       */
  int pose_chunk;            /* poses per selection-net launch (its per-pose    */
                             /* intermediates take (51 n + 8 n_tets) doubles    */
                             /* each); 0: automatic, every pose up to 4 GiB of  */
                             /* them.  Results do not depend on it              */
} nmr_cubature_train_desc;

/* Neural cubature training (Sec. 5) on the instance's mesh, decoder and U:
 * computes the training data of every pose (nmr_element_forces) into device
 * memory (P x n_tets x R doubles of element forces, the run's largest
 * buffer), copies both nets and picks the initial set.  The trainer keeps no
 * reference to the instance.  NMR_ERR_INVERTED if a pose inverts a tet;
 * NMR_ERR_BUDGET beyond the context's HBM budget.  Synchronizes. */
int nmr_trainer_create(nmr_inst* inst, const nmr_cubature_train_desc* desc, nmr_trainer** out);
int nmr_trainer_destroy(nmr_trainer* tr);

/* n_alternations alternations of Sec. 5: `epochs` full-batch Adam steps of
 * the weight net on L_W = mean_p |f_p - sum_{j<|C|} w_j(r_p) F_p[C_j]|^2 /
 * |f_p|^2; the residual forces fb_p of the trained weights (eq. of the
 * residual force); `epochs` Adam steps of the selection net -- two graph
 * convolutions h' = sin(sum over the one-ring (self included) of
 * h_j Gamma / sqrt(d_i d_j)) of the vertex displacements, element feature =
 * mean of its vertices, sin(A1 g + a1), logit A2 . y + a2, scores e^c times
 * the softmax over the elements outside C -- on L_S = mean_p |fb_p -
 * sum_{e not in C} s_e F_p[e]|^2 / |fb_p|^2; then the K elements outside C
 * with the largest score averaged over the poses (ties to the lower id) join
 * C.  Each net keeps its Adam state across alternations; rows of the weight
 * net's last layer beyond |C| stay as given until their element joins.
 * Host outputs (each may be NULL): loss_w and loss_s [n_alternations x
 * epochs], each net's loss before each of its steps; added [n_alternations x
 * K]; ms_or_null: device time of the whole call.  NMR_ERR_ARG if |C| would
 * exceed c_max.  Every sum runs in a fixed order: a run is bitwise repeatable.
 * Synchronizes. */
int nmr_trainer_run(nmr_trainer* tr, int n_alternations, double* loss_w, double* loss_s, int* added,
                    float* ms_or_null);

/* The current set and nets (host outputs, each but n_c may be NULL): n_c =
 * |C|, C [|C|] in joining order, the weight net's parameters [W_0 (row-major),
 * b_0, ..., W_{L-1} (c_max rows), b_{L-1}] and the 170 selection-net
 * parameters.  The first |C| rows of the last layer with scale wnet_scale
 * form the run-time weight net of an instance whose cubature set is C. */
int nmr_trainer_get(nmr_trainer* tr, int* n_c, int32_t* C_or_null, double* wnet_or_null, double* snet_or_null);

/* Training data of pose p (host outputs, each may be NULL): F [n_tets x R],
 * f [R], u [N]. */
int nmr_trainer_pose(nmr_trainer* tr, int p, double* F_or_null, double* f_or_null, double* u_or_null);

/* Pieces of an alternation, for measurement. */
typedef enum {
  NMR_TRAIN_PHASE_S_EPOCH = 0,    /* one selection-net epoch without its Adam step */
  NMR_TRAIN_PHASE_W_EPOCH = 1,    /* one weight-net epoch without its Adam step    */
  NMR_TRAIN_PHASE_S_ELEM_FWD = 2, /* the selection net's element forward pass      */
  NMR_TRAIN_PHASE_S_ELEM_BWD = 3, /* the selection net's element backward pass     */
  NMR_TRAIN_PHASE_COUNT = 4
} nmr_train_phase;

/* Replays one phase `reps` times on the context stream between two HIP
 * events (after the residual forces and a forward pass that give it valid
 * inputs, and one untimed replay) and writes the mean device time per replay
 * in microseconds to *avg_us (host).  Only intermediates are written: the
 * nets, their Adam states and the cubature set are unchanged.  Synchronizes. */
int nmr_trainer_time_phase(nmr_trainer* tr, int phase, int reps, float* avg_us);

/* ---- measurement -------------------------------------------------------- */

/* Phases of one Newton iteration, in launch order. */
typedef enum {
  NMR_PHASE_DEC_HIDDEN = 0, /* forward jet GEMMs of the hidden layers         */
  NMR_PHASE_DEC_OUT = 1,    /* output-layer GEMM (+ filter when n_p > 0)      */
  NMR_PHASE_CUBATURE = 2,   /* cubature force / reduced stiffness             */
  NMR_PHASE_MASS = 3,       /* mass terms, residual pieces, BP seed           */
  NMR_PHASE_SUMS = 4,       /* fixed-order sums of the partials               */
  NMR_PHASE_BWD_OUT = 5,    /* backpropagation through the output layer       */
  NMR_PHASE_BWD_HIDDEN = 6, /* partial-sum reduce + hidden-layer complex BP   */
  NMR_PHASE_SOLVE = 7,      /* assemble, LU solve, update                     */
  NMR_PHASE_COUNT = 8
} nmr_phase;

/* Replays one phase of a Newton iteration of `inst` `reps` times on the
 * context stream between two HIP events (after one untimed replay) and
 * writes the mean device time per replay in microseconds to *avg_us (host).
 * The instance state is saved before and restored after, so the call does
 * not change the trajectory.  Synchronizes. */
int nmr_time_phase(nmr_inst* inst, int phase, int reps, float* avg_us);

#ifdef __cplusplus
}
#endif
#endif /* NMR_H */
