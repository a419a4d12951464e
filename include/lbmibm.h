/*
 * lbmibm.h -- C ABI of the MI355X (gfx950) LBM-IBM library.
 *
 * The library advances a D3Q19 BGK lattice-Boltzmann fluid with a body-force
 * term (Beny & Latt, arXiv 1904.02108, §2: eqs. (1)-(4) and the six-step
 * time loop) and computes that force with the multi-direct-forcing immersed
 * boundary method of Ota, Suzuki and Inamuro (§3: interpolation through
 * Peskin's 4-point delta, deficit g(k), accumulated correction du(k),
 * intermediate spreading, final spreading into G; §4.2-4.3: Algorithms 1
 * and 2) for rigidly rotating Lagrangian surfaces.
 *
 * Conventions shared by every call
 *   - Every function returns lbm_status (0 = LBM_OK, < 0 = error).  No C++
 *     exception crosses the ABI.  After an error, lbm_last_error(ctx) holds a
 *     message; the context is unchanged except after LBM_ERR_HIP, after which
 *     it must be destroyed.
 *   - Work is enqueued on the stream given in lbm_params (a hipStream_t,
 *     borrowed, never destroyed by the library; NULL = the null stream).
 *     Calls return before the GPU finishes unless a host pointer is read or
 *     written, or a stats/residual result is requested.
 *   - Large device memory is owned by the caller: lbm_buffer_sizes() gives
 *     the byte size of each buffer, the caller allocates them (any device
 *     allocator; 256-byte alignment) and passes them to lbm_create(); they
 *     must outlive the context.  The library owns only host metadata.
 *   - A context is not thread-safe; calls on one context must be serialised.
 *   - Lattice units: cell X sits at integer coordinates 0..n-1 on each axis;
 *     dx = dt = 1.  Fields are exported x-fastest: index x + nx*(y + ny*z).
 *   - D3Q19 direction order (POPS export): 0 rest; 1..6 = +x,-x,+y,-y,+z,-z;
 *     7..18 = (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),
 *     (1,0,-1),(-1,0,1),(0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1).
 */
#ifndef LBMIBM_H
#define LBMIBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque context: one simulation on one device. */
typedef struct lbm_ctx lbm_ctx;

typedef int32_t lbm_status;
enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,       /* invalid argument (sizes, pointers, enums)        */
  LBM_ERR_OOM = -2,       /* a caller buffer is missing or too small          */
  LBM_ERR_HIP = -3,       /* a HIP runtime call or launch failed              */
  LBM_ERR_STATE = -4,     /* call not valid in the current state              */
  LBM_ERR_DOMAIN = -5,    /* a point's kernel support leaves a walled box     */
  LBM_ERR_NONFINITE = -6  /* non-finite state detected (see lbm_set_check)     */
};

/* Boundary condition per axis (both faces).  Bounce-back is the halfway
 * rule: walls half a cell outside the first and last cell. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_BOUNCEBACK = 1 };

/* Population storage in HBM.  All arithmetic is FP32; the 16-bit forms store
 * f_i - t_i (offset from the lattice weight), rounded to nearest even. */
enum { LBM_STORE_F32 = 0, LBM_STORE_F16 = 1, LBM_STORE_BF16 = 2 };

/* Forcing scheme for the force G (an acceleration) in the collision:
 *   GUO:   F = rho G, equilibrium at U + G/2, plus Guo's source term;
 *   SHIFT: the paper's velocity shift, equilibrium at U + tau G (§2, step 3).
 * Both change the momentum by exactly rho G per step. */
enum { LBM_FORCE_GUO = 0, LBM_FORCE_SHIFT = 1 };

typedef struct {
  int32_t nx, ny, nz;      /* lattice size, each >= 1                          */
  int32_t bc[3];           /* LBM_BC_* per axis                                */
  int32_t storage;         /* LBM_STORE_*                                      */
  int32_t forcing;         /* LBM_FORCE_*                                      */
  double tau;              /* BGK relaxation time, > 0.5                       */
  double rho_wall;         /* density in the moving-wall correction (Ladd)     */
  double wall_u[3][2][3];  /* wall velocity [axis][0 = low, 1 = high face][c]  */
  double g_ext[3];         /* uniform acceleration added to G in every cell    */
  double rho0;             /* initial uniform density                          */
  double u0[3];            /* initial uniform velocity                         */
  int64_t max_points;      /* capacity for Lagrangian points (>= 0)            */
  int32_t max_iter;        /* capacity for forcing sweeps per step (1..64)     */
  int32_t reserved_;       /* must be 0                                        */
  void* stream;            /* hipStream_t, borrowed                            */
} lbm_params;

/* Caller-owned device buffers. */
enum {
  LBM_BUF_LATTICE = 0,  /* two population lattices                        */
  LBM_BUF_FIELDS = 1,   /* velocity scratch U and force G, 3 x FP32 each  */
  LBM_BUF_POINTS = 2,   /* Lagrangian point arrays                        */
  LBM_BUF_TILES = 3,    /* tile counts, offsets, flags                    */
  LBM_BUF_SCRATCH = 4,  /* reduction partials and small results           */
  LBM_NBUF = 5
};

/* Rigid body: rotation about `axis` (normalised by the library) through
 * `center`, by theta_n = theta0 + omega * n at time step n (§4.2: the motion
 * M(t) is applied to the rest positions at the first sweep). */
typedef struct {
  double center[3];
  double axis[3];
  double theta0;
  double omega;
} ibm_body;

/* ibm_set_points flags */
enum {
  IBM_INNER_UNWEIGHTED = 1u, /* spread g(k) (not s(k) g(k)) inside the sweep,
                                the paper-literal reading of §3             */
  IBM_STOP_RESIDUAL = 2u,    /* sweep until the relative boundary-velocity
                                residual R_rel <= eps, at most n_iter sweeps
                                (§3 notes the sweeps could run until the
                                deficit is negligible); the sweep that meets
                                the threshold applies its correction and
                                spreads du into G, as the last fixed sweep
                                does.  R_rel = sqrt(sum s|g|^2 / sum s|u_b|^2)
                                of the deficit g of a sweep (tested as
                                sum s|g|^2 <= eps^2 sum s|u_b|^2, so a body at
                                rest converges).  Decided on the device: the
                                launches of later sweeps return at once, with
                                no host synchronisation.                     */
  IBM_WARM_START = 4u,       /* learned warm start (not in the paper): before
                                the first correction, an MLP set with
                                ibm_set_mlp predicts du from the first deficit
                                g0, u_b and the mean and component-wise max of
                                g0 over the point's neighbours, all divided by
                                the body's reference speed; the prediction is
                                spread into U and the sweeps continue from it.
                                Useful with IBM_STOP_RESIDUAL, valid alone;
                                not with IBM_INNER_UNWEIGHTED or
                                IBM_WARM_PREV.                               */
  IBM_KEEP_FEATURES = 8u,    /* compute the features in every forcing so that
                                ibm_log_pairs can export training pairs       */
  IBM_MLP_FP32 = 16u,        /* evaluate the warm-start network with FP32
                                weights and activations (FP32 operands on the
                                matrix cores); default: BF16 operands on the
                                matrix cores; both accumulate in FP32         */
  IBM_WARM_PREV = 32u,       /* warm start from the previous forcing (not in
                                the paper; the non-learned baseline of
                                IBM_WARM_START): after the first deficit g0,
                                the final du of the same point in the last
                                forcing replaces s g0, is spread into U and
                                the sweeps continue from it.  The first
                                forcing after ibm_set_points or a write of
                                LBM_F_POPS has no previous du and runs the
                                plain first sweep.  Not with IBM_WARM_START. */
  IBM_U_BOX = 64u,           /* U pre-pass (§5) by the box strategy: U on every
                                cell of each body's bounding box, the rest-
                                position box of its points moved by the step's
                                rigid motion, widened by the kernel support   */
  IBM_U_KERNEL = 128u        /* U pre-pass by the kernel strategy (§5): U on
                                the 4^3 support cells of every point (cells
                                shared by several supports are computed once
                                per point).  Default (neither bit): U on the
                                4^3 blocks that some support reaches.  All
                                three give the same U wherever it is read, so
                                the results are identical; only the time
                                differs.  Not both.                          */
};

/* mlp_forward precision */
enum { MLP_FP32 = 0, MLP_BF16 = 1 };

/* Learned warm start: a per-point MLP 12 -> 64 -> 64 -> 64 -> 3 with SiLU
 * after each hidden layer.  Flat FP32 parameter layout (row-major, out x in):
 *   W1[64][12] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3].
 * Features of point k (in this order, each divided by the reference speed
 * v_ref of k's body = |omega| * max_j |r_j| over the body's rest points, or
 * 1 for a body at rest): g0 (3), u_b (3), mean of g0 over N(k) (3),
 * component-wise max of g0 over N(k) (3), zeros when N(k) is empty.
 * N(k): up to 16 points of k's body nearest to k at Euclidean distance < 2,
 * ordered by (distance, index).  Distances are those of the rest positions,
 * computed in FP64 as ((dx^2 + dy^2) + dz^2) with every operation rounded,
 * so N(k) is exact, fixed for a rigid body, and found once per surface.
 * Output y: du = s(k) v_ref y, so the training target is du / (s v_ref)
 * (0 where s = 0). */
#define IBM_MLP_NPARAM 9347
#define IBM_MLP_NFEAT 12
#define IBM_MLP_NNBR 16

#define LBM_MAX_ITER 64

/* Per-step forcing statistics (FP64 sums over points). */
typedef struct {
  int32_t n_iter;                /* sweeps executed                         */
  int32_t pad_;
  double sum_s;                  /* sum_k s(k)                              */
  double sum_s_ub2;              /* sum_k s(k) |u_b(k)|^2                   */
  double resid[LBM_MAX_ITER];    /* sum_k s(k) |g_it(k)|^2 for each sweep   */
} ibm_stats;

/* lbm_read_fields / lbm_write_fields masks */
enum {
  LBM_F_RHO = 1u << 0,   /* float [nz][ny][nx]      density (read)            */
  LBM_F_VEL = 1u << 1,   /* float [3][nz][ny][nx]   U = sum e f / rho (read)  */
  LBM_F_FORCE = 1u << 2, /* float [3][nz][ny][nx]   G of the last forcing;
                            write: prescribes G (only without points)        */
  LBM_F_POPS = 1u << 3,  /* float or double [19][nz][ny][nx] populations f
                            at the start of the current step (after stream)  */
  LBM_F_PT_X = 1u << 4,  /* double [n][3] point positions of the last forcing */
  LBM_F_PT_UB = 1u << 5, /* float  [n][3] point velocities u_b                */
  LBM_F_PT_G = 1u << 6,  /* float  [n][3] last deficit g                      */
  LBM_F_PT_DU = 1u << 7, /* float  [n][3] accumulated correction du           */
  LBM_F_SUMS = 1u << 8,  /* double [4]   sum rho, sum rho U over the box at the
                            start of the last completed step                 */
  LBM_F_STEP = 1u << 9   /* int64  [1]   current time step index              */
};

typedef struct {
  int32_t on_device;   /* 1: device pointers (async on the stream);
                          0: host pointers (the call synchronises; the
                          data pass through a device staging buffer that
                          the context allocates once, grows to the largest
                          request and keeps until lbm_destroy)              */
  int32_t pops_f64;    /* POPS as double (1) or float (0)                     */
  float* rho;
  float* vel;
  float* force;
  void* pops;
  double* pt_x;        /* point arrays are in the order given to ibm_set_points */
  float* pt_ub;
  float* pt_g;
  float* pt_du;
  double* sums;
  int64_t* step;
} lbm_fields;

/* Byte sizes of the LBM_NBUF caller buffers for these parameters. */
lbm_status lbm_buffer_sizes(const lbm_params* p, size_t sizes_out[LBM_NBUF]);

/* Creates a context on the current HIP device, binds the caller buffers and
 * enqueues the initial state f = Eq(rho0, u0) at step 0.  The buffers are
 * not read before this call and need no initialisation. */
lbm_status lbm_create(const lbm_params* p, void* const bufs[LBM_NBUF], lbm_ctx** out);

/* Destroys the context and the device staging buffer of host-pointer
 * field reads and writes; the caller frees its buffers. */
void lbm_destroy(lbm_ctx* ctx);

/* Last error message of ctx, or of the last failed lbm_create or
 * mlp_loss_grad_noalloc on this thread when ctx is NULL.  Valid until the
 * next call on the context. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Sets the immersed surface (§3, §4.2): n points with rest positions
 * relative to their body's centre (host float [n][3]), areas s(k) (host
 * float [n]), body ranges body_off[0..nbodies] (host, body b owns points
 * body_off[b] .. body_off[b+1]-1, body_off[0] = 0, body_off[nbodies] = n),
 * bodies (host [nbodies]), n_iter sweeps per step (1..max_iter), flags
 * (IBM_*), eps (see below).  Host arrays are copied before return.
 * n = 0 removes the surface.  eps: residual threshold for
 * IBM_STOP_RESIDUAL (else must be 0).  Returns LBM_ERR_DOMAIN if for some
 * rotation angle a support could leave a walled axis (bounding-sphere test:
 * on a bounce-back axis every point must keep 1 <= x < n - 2). */
lbm_status ibm_set_points(lbm_ctx* ctx, int64_t n, const float* rest_xyz, const float* area,
                          const int64_t* body_off, int32_t nbodies, const ibm_body* bodies,
                          int32_t n_iter, uint32_t flags, float eps);

/* Computes the force G for the current step (§2 step 2, §3): moves the
 * points (Algorithm 1), computes U near them, runs the sweeps and spreads
 * du into G.  A following lbm_step uses this G instead of recomputing it.
 * stats (nullable; non-NULL synchronises the stream) receives the sums. */
lbm_status ibm_force_iterate(lbm_ctx* ctx, ibm_stats* stats);

/* Advances n_steps >= 0 time steps: per step, the forcing (if a surface is
 * set) followed by the fused stream-collide (§2 steps 1, 3-6). */
lbm_status lbm_step(lbm_ctx* ctx, int32_t n_steps);

/* Failure detection (not in the paper): the stream-collide raises a sticky
 * device status word when a workgroup's FP64 partial of the mass or
 * momentum sums is not finite (a NaN or infinite population, §2 eq. (1)),
 * and a forcing sweep raises another when a value it spreads (§3, Algorithm
 * 2) is not finite or exceeds 4096 in magnitude, beyond which the spread's
 * fixed-point accumulation cannot represent it.  every > 0: lbm_step
 * synchronises after every `every` steps, and ibm_force_iterate after each
 * forcing, reads the words and returns LBM_ERR_NONFINITE if one is raised
 * (lbm_last_error names which and the step reached).  The steps before the
 * check have run and are not undone; the words stay raised until the next
 * lbm_set_check.  every = 0 (the default) turns the check off; the words are
 * raised either way.  Each call clears them.  LBM_ERR_ARG for every < 0. */
lbm_status lbm_set_check(lbm_ctx* ctx, int32_t every);

/* Reads fields selected by mask into caller memory (see LBM_F_*). */
lbm_status lbm_read_fields(lbm_ctx* ctx, uint32_t mask, const lbm_fields* dst);

/* Writes LBM_F_POPS (f at the start of the current step), LBM_F_FORCE
 * (prescribed G, kept until the next write, only without points) and
 * LBM_F_STEP.  Other bits are rejected with LBM_ERR_ARG. */
lbm_status lbm_write_fields(lbm_ctx* ctx, uint32_t mask, const lbm_fields* src);

/* Learned warm start: sets the MLP parameters (host float [IBM_MLP_NPARAM],
 * copied before return). */
lbm_status ibm_set_mlp(lbm_ctx* ctx, const float* theta);

/* Training pairs of the last forcing (after ibm_force_iterate or lbm_step)
 * of a surface set with IBM_KEEP_FEATURES: features
 * [n][12] (those of the first sweep) and the target du / (s v_ref) [n][3]
 * of the final correction du, in the order given to ibm_set_points, into
 * caller device memory (enqueued on the context's stream).  LBM_ERR_STATE
 * without such a forcing. */
lbm_status ibm_log_pairs(lbm_ctx* ctx, float* features, float* targets);

/* Statistics of the last forcing: sweeps run, sum s, sum s |u_b|^2 and the
 * residual sum s |g|^2 of each sweep (synchronises). */
lbm_status ibm_last_stats(lbm_ctx* ctx, ibm_stats* stats);

/* Stateless MLP kernels on caller device memory, enqueued on `stream`:
 *   mlp_forward:   y[n][3] = MLP(theta; x[n][12]) in FP32 (precision
 *                  MLP_FP32, workspace may be NULL) or with BF16 operands
 *                  and FP32 accumulation on the matrix cores (MLP_BF16,
 *                  workspace of at least mlp_workspace_size(1) bytes);
 *   mlp_loss_grad: loss = (1 / 3n) sum (y - t)^2 into loss_out (device
 *                  double[1]) and its gradient into grad (device float
 *                  [IBM_MLP_NPARAM]);
 *   mlp_train:     n_epochs passes of Adam (beta1 0.9, beta2 0.999, eps 1e-8)
 *                  over mini-batches of `batch` consecutive pairs, on theta in
 *                  place; m, v: device float [IBM_MLP_NPARAM] Adam moments
 *                  (zero them before the first call), *step_t: Adam step
 *                  count (host, in/out); loss_per_epoch (host, nullable,
 *                  [n_epochs]): mean batch loss of each epoch (synchronises).
 * workspace: device memory of mlp_workspace_size(batch) bytes. */
size_t mlp_workspace_size(int64_t batch);
lbm_status mlp_forward(const float* theta, int64_t n, const float* x, float* y,
                       int32_t precision, void* workspace, void* stream);
lbm_status mlp_loss_grad(const float* theta, int64_t n, const float* x, const float* t,
                         float* grad, double* loss_out, void* workspace, void* stream);
lbm_status mlp_train(float* theta, float* m, float* v, int64_t* step_t, int64_t n,
                     const float* x, const float* t, int64_t batch, int32_t n_epochs,
                     double lr, double* loss_per_epoch, void* workspace, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): mlp_loss_grad
 * with the library's own workspace instead of a caller one.  The workspace
 * is a fixed device array held by the library (about 2.7 MB on each device
 * it runs on, until the process ends), sized for n <= MLP_NOALLOC_MAX_BATCH
 * samples; a larger n returns LBM_ERR_ARG (message in lbm_last_error(NULL)).
 * The call allocates nothing (no hipMalloc, no allocating library routine);
 * its first call on a device looks up the array's device address there.
 * Arguments, layouts and results as mlp_loss_grad: theta, x [n][12], t [n][3],
 * grad [IBM_MLP_NPARAM] and loss_out (nullable, double[1]) are caller device
 * memory; work is enqueued on `stream`.  Every call on a device shares that
 * device's workspace, which keeps the last call's contents (each call writes
 * every byte it reads first): calls that overlap on one device, on different
 * streams or threads, race and must be serialised by the caller. */
#define MLP_NOALLOC_MAX_BATCH 1024
lbm_status mlp_loss_grad_noalloc(const float* theta, int64_t n, const float* x, const float* t,
                                 float* grad, double* loss_out, void* stream);

/* Optional per-phase timing with HIP events on the context's stream.
 * lbm_get_timing returns {ms forcing, ms stream-collide, forcing calls,
 * stream-collide calls} accumulated since enabling, and synchronises. */
lbm_status lbm_set_timing(lbm_ctx* ctx, int32_t enable);
lbm_status lbm_get_timing(lbm_ctx* ctx, double out[4]);

#ifdef __cplusplus
}
#endif
#endif /* LBMIBM_H */
