/*
 * ppd.h -- C ABI of libppd, a gfx950 (MI355X) implementation of the
 * per-iteration hot path of the preconditioned primal-dual (PPD) imager of
 * Onose, Dabbech & Wiaux (2017), "An accelerated splitting algorithm for
 * radio-interferometric imaging: when natural and uniform weighting meet".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers are DEVICE pointers unless the comment says HOST.  The caller
 * owns every buffer it passes; the library owns only the plan and the
 * device memory the plan allocates at creation (freed by ppd_plan_destroy).
 * All launches are asynchronous on the plan's stream (see
 * ppd_plan_set_stream); entry points that return host values synchronise
 * that stream and say so.  Arguments are validated on the host before any
 * launch, so a non-zero status leaves every output untouched.  A plan is not
 * thread safe: use one plan per stream.  No exception crosses the ABI.
 *
 * Layouts: an image is ny rows x nx columns, row-major, float32; row r is
 * the v axis, column c the u axis, pixel (ny/2, nx/2) is the phase centre.
 * Complex arrays are interleaved (re, im): complex64 = 2 x float32,
 * complex128 = 2 x float64.  SARA coefficient / dual arrays are
 * [9][ny][nx] float32, basis 0 = Dirac, basis p = Daubechies-p (p = 1..8),
 * each basis in the Mallat pyramid layout of the image size.
 *
 * Visibility order: per-visibility arrays are indexed in PLAN order by
 * default -- the visibilities of each data block stay inside that block's
 * range [block_off[j], block_off[j+1]) but are re-ordered by grid tile.
 * ppd_plan_permutation / ppd_plan_permute convert from and to USER order
 * (the order of omega_u / omega_v at plan creation).
 */
#ifndef PPD_H
#define PPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PPD_OK            0
#define PPD_EINVAL       -1   /* bad argument; nothing was launched          */
#define PPD_ENOMEM       -2   /* device allocation failed at plan creation   */
#define PPD_EDEVICE      -3   /* a HIP runtime call failed                   */
#define PPD_ENONFINITE   -4   /* iteration statistics became NaN or Inf      */
#define PPD_EUNSUPPORTED -5   /* valid but not implemented (e.g. sizes)      */

/* Human-readable text for a status code (static storage). */
const char* ppd_strerror(int status);
/* Text of the last error raised on this thread (static per thread). */
const char* ppd_last_error(void);

/* ---- plan -------------------------------------------------------------- */
typedef struct ppd_plan ppd_plan;

typedef struct {
  int32_t nx, ny;             /* image size; powers of two, 16 <= n <= 2048,
                                 divisible by 2^levels                          */
  int64_t M;                  /* number of visibilities, 1 <= M < 2^31          */
  int32_t d;                  /* number of data blocks y_j (Sec. 3.1), >= 1     */
  const int64_t* block_off;   /* HOST [d+1], 0 = off[0] < off[1] < .. = M       */
  const float* omega_u;       /* HOST [M] u frequencies, rad/pixel in [-pi, pi) */
  const float* omega_v;       /* HOST [M] v frequencies, rad/pixel in [-pi, pi) */
  const float* theta;         /* HOST [M] natural weights 1/sigma_e (Sec. 2), or
                                 NULL for theta = 1                              */
  double kb_beta;             /* Kaiser-Bessel shape; <= 0 selects the default
                                 pi sqrt(35.2) (width 8, 2x oversampling)        */
  int32_t levels;             /* SARA decomposition levels (1..6), 0 -> 3       */
  int32_t tile;               /* gridding tile edge in grid cells: 8, 16, 32 or
                                 64 (8: gridding on the matrix cores); 0 -> 8    */
  int32_t chunk;              /* max visibilities per work chunk (64..65536),
                                 0 -> 128 for tile 8, else 512; a chunk also
                                 holds at most 64 data blocks' segments of its
                                 tile                                            */
} ppd_plan_desc;

/* Create a plan: validates desc, bins the visibilities by (block, tile) on
 * the host, uploads the sorted coverage, Kaiser-Bessel polynomial
 * coefficients, deapodisation factors, FFT twiddles and Daubechies filters,
 * and allocates the plan's work buffers.  Synchronous.  `stream` is a
 * hipStream_t (NULL = default stream) used by every later call. */
int ppd_plan_create(ppd_plan** plan, const ppd_plan_desc* desc, void* stream);

/* The same plan with every device buffer carved from a caller-owned
 * workspace, so that the caller's allocator (PyTorch) is the only one.
 * ppd_plan_workspace_size runs the host part of plan creation (validation
 * and binning, no HIP call) and returns the bytes needed; ppd_plan_create_ws
 * takes a DEVICE workspace of at least that size, 256-byte aligned, which
 * must stay allocated and untouched until ppd_plan_destroy (which does not
 * free it).  Errors: PPD_EINVAL for a NULL, misaligned or too small
 * workspace, else as ppd_plan_create. */
int ppd_plan_workspace_size(const ppd_plan_desc* desc, size_t* bytes /* HOST */);
int ppd_plan_create_ws(ppd_plan** plan, const ppd_plan_desc* desc, void* workspace, size_t bytes,
                       void* stream);
int ppd_plan_destroy(ppd_plan* plan);
int ppd_plan_set_stream(ppd_plan* plan, void* stream);

typedef struct {
  int32_t nx, ny, Kx, Ky;     /* image and oversampled grid sizes (K = 2 n)     */
  int64_t M;
  int32_t d, levels, tile, chunk;
  int32_t n_chunks;           /* work chunks (one workgroup each)               */
  double kb_beta;
  size_t device_bytes;        /* device memory of the plan's buffers (allocated,
                                 or carved from the caller's workspace)         */
  int32_t persistent;         /* 1 if the Algorithm 2 middle steps can run as
                                 one persistent launch (ppd_params.persistent) */
  int32_t pad_;
} ppd_plan_info;
int ppd_plan_get_info(const ppd_plan* plan, ppd_plan_info* info /* HOST */);

/* perm[p] = user index of plan position p.  HOST [M] int64.  Synchronous. */
int ppd_plan_permutation(const ppd_plan* plan, int64_t* perm /* HOST */);

#define PPD_USER_TO_PLAN 0
#define PPD_PLAN_TO_USER 1
/* Re-order a per-visibility device array (elem_bytes in {4, 8, 16}). */
int ppd_plan_permute(ppd_plan* plan, int direction, const void* in, void* out, int elem_bytes);

/* ---- measurement operator (Sec. 2: Phi = Theta G F Z) ------------------ */
#define PPD_ORDER_PLAN 0
#define PPD_ORDER_USER 1

/* y = Theta G F Z x (Sec. 2): Kaiser-Bessel 8x8 degridding of the 2x
 * oversampled, deapodised FFT of the image.  x: [ny][nx] float32.
 * y: [M] complex64 in the given order. */
int ppd_phi(ppd_plan* plan, const float* x, float* y, int order);

/* x = Re(Z^H F^H G^H Theta^H y), the adjoint of ppd_phi for a real image
 * (Sec. 2; the gridding and the primal step of Algorithm 3).
 * y: [M] complex64 in the given order.  x: [ny][nx] float32. */
int ppd_phit(ppd_plan* plan, const float* y, float* x, int order);

/* ---- SARA sparsity operator (Sec. 5.1: Dirac + Daubechies 1..8) -------- */
#define PPD_SARA_ANALYSIS  0   /* out[9][ny][nx] = Psi^H in  (in: image)        */
#define PPD_SARA_SYNTHESIS 1   /* out[ny][nx] = Psi in       (in: [9][ny][nx])  */
#define PPD_SARA_DUAL      2   /* SARA dual update of Algorithm 3, W = I:
                                  u <- u + lambda (clip(u + Psi^H in, +-alpha) - u),
                                  out[ny][nx] = Psi u  (in: image, u_inout used) */
/* Psi = (1/3)[I, W_1, .., W_8] with W_p the orthonormal periodised 2D
 * Daubechies-p DWT, so Psi Psi^H = I.  u_inout may be NULL unless op is
 * PPD_SARA_DUAL.  (I - S_alpha) is the soft-threshold complement of
 * Sec. 3.3, i.e. a clip to [-alpha, alpha]. */
int ppd_sara(ppd_plan* plan, int op, const float* in, float* out, float* u_inout,
             float alpha, float lambda);

/* ppd_sara with per-coefficient re-weights W ([9][ny][nx], Sec. 3.2 and
 * Algorithm 1; NULL = identity): analysis gives W Psi^H in, synthesis
 * Psi W in, and the dual mode clips u + W Psi^H in and returns Psi W u. */
int ppd_sara_w(ppd_plan* plan, int op, const float* in, float* out, float* u_inout,
               const float* W, float alpha, float lambda);

/* Re-weights of Algorithm 1 (eq. reweighting, Sec. 3.2):
 * W_i = omega / (omega + |Psi_i^H x|) per coefficient, for the image x
 * ([ny][nx]); W: [9][ny][nx] float32 output.  omega > 0. */
int ppd_reweight(ppd_plan* plan, const float* x, float omega, float* W);

/* ---- data-fidelity dual: ellipsoid projection (Sec. 4.1, Algorithm 2) -- */
/* n_itr forward-backward iterations, per block j,
 *     z <- P_B(z - mu U (z - w)),   P_B the projection onto
 *     {z : ||z - y_j||_2 <= eps_j},
 * approximating prox^U_h(w) of eq. elip-proj-1.  FP64 arithmetic and
 * block norms.  w, zbar_inout: [M] complex128; y: [M] complex64;
 * U: [M] float64 > 0; eps: HOST [d] float64 > 0; mu > 0.  Plan order. */
int ppd_ellipsoid_proj(ppd_plan* plan, const double* w, const float* y, const double* U,
                       const double* eps, int n_itr, double mu, double* zbar_inout);

/* ppd_ellipsoid_proj for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same n_itr Algorithm 2 iterations per block, with no plan
 * and no allocation of any kind.  Block j is the contiguous range
 * [block_off[j], block_off[j+1]) of the arrays (any order inside a block,
 * e.g. a plan's order); w, zbar_inout: [M] complex128; y: [M] complex64;
 * U: [M] float64 > 0 (DEVICE, M = block_off[d]); block_off: HOST [d+1]
 * int64, 0 = off[0] < off[1] < ...; eps: HOST [d] float64 > 0; mu > 0;
 * stream: hipStream_t (NULL = default stream).  Limits: d <= 4096 and at
 * most 65536 chunks of 8192 points (about 5.4e8 visibilities); beyond them
 * PPD_EINVAL and nothing is launched.  The per-block partial sums and
 * factors live in one fixed device array of about 0.7 MiB that each GPU the
 * library runs on holds until the process ends; every call on a GPU uses
 * that GPU's array, so calls that overlap on one GPU (on different streams
 * or host threads) race and must be ordered by the caller.  Asynchronous on
 * `stream` (the host tables are staged by the runtime before it returns). */
int ppd_ellipsoid_proj_noalloc(const double* w, const float* y, const double* U, int32_t d,
                               const int64_t* block_off, const double* eps, int n_itr, double mu,
                               double* zbar_inout, void* stream);

/* The prox of eq. elip-proj-1 itself (the exact alternative the paper
 * names next to Algorithm 2, Sec. 4.1): per block j,
 *     z = argmin_{||z - y_j|| <= eps_j} (w - z)^H U_j (w - z) / 2
 *       = (U w + nu_j y) / (U + nu_j),
 * nu_j = 0 if ||w - y_j|| <= eps_j, else the root of ||U (w - y_j) / (U + nu)||
 * = eps_j, found by n_newton Newton steps on 1 / ||.|| - 1 / eps_j from
 * nu = 0 (concave and increasing in nu, so the steps approach the root
 * monotonically from below).  FP64.  w, z: [M] complex128 (z may alias
 * nothing else); y: [M] complex64; U: [M] float64 > 0; eps: HOST [d];
 * nu: optional DEVICE [d] float64 output.  1 <= n_newton <= 64.  Plan order. */
int ppd_prox_metric(ppd_plan* plan, const double* w, const float* y, const double* U,
                    const double* eps, int n_newton, double* z, double* nu);

/* ---- setup quantities (Sec. 4.3, Sec. 5.1) ------------------------------ */
/* Uniform-weighting preconditioner: the inverse sampling density near each
 * visibility.  Points are counted on an ny x nx u-v cell grid, cell
 * floor((omega + pi) n / (2 pi)) clamped to n - 1; U_e = c_min / c_e so that
 * max U = 1.  U: [M] float64, plan order. */
int ppd_uniform_weights(ppd_plan* plan, double* U);

/* ||U^1/2 Phi||_S^2 by power iteration on x -> Re Phi^H (U Phi x) from the
 * start image x0 ([ny][nx] float32; not modified); U may be NULL (U = 1).
 * Stops when the relative change of the estimate is <= tol or after
 * max_iter iterations.  Synchronous; result in *norm2 (HOST). */
int ppd_op_norm(ppd_plan* plan, const double* U, const float* x0, int max_iter, double tol,
                double* norm2, int* iters);

/* ---- Algorithm 3 (PPD) -------------------------------------------------- */
typedef struct {
  float* x;        /* [ny][nx] primal image x                                 */
  float* xt;       /* [ny][nx] x tilde                                        */
  float* v;        /* [M] complex64 data duals v_j (plan order)               */
  float* u;        /* [9][ny][nx] sparsity duals u_i                          */
  double* z;       /* [M] complex128 Algorithm 2 iterate (warm start)         */
  int64_t iter;    /* iterations done; advanced by ppd_iterate                */
} ppd_state;

#define PPD_FORM_FUSED 0   /* one launch per step for all blocks, dual update
                              fused into (de)gridding, FP64 projection        */
#define PPD_FORM_PLAIN 1   /* unfused reference form: Phi, per-block FP64
                              dual kernels, Phi^H, each a separate launch     */

#define PPD_PROX_FB    0   /* prox^U_h by n_itr Algorithm 2 iterations        */
#define PPD_PROX_EXACT 1   /* prox^U_h exactly (ppd_prox_metric, n_newton
                              Newton steps); fused form only                  */

#define PPD_PERSIST_AUTO 0
#define PPD_PERSIST_OFF  1

typedef struct {
  double tau, eta, zeta, lambda;   /* Algorithm 3 step sizes and relaxation   */
  double alpha;                    /* l1 dual clip kappa ||Psi W||_S^2        */
  double mu;                       /* Algorithm 2 step, <= 1 / max U          */
  int32_t n_itr;                   /* Algorithm 2 iterations (>= 1)           */
  int32_t form;                    /* PPD_FORM_*                              */
  int32_t use_graph;               /* replay one captured iteration as a HIP
                                      graph (needs a non-default plan stream);
                                      re-captured when a pointer or scalar of
                                      these params or the state changes      */
  int32_t pad_;
  const float* y;                  /* [M] complex64 data, plan order          */
  const double* U;                 /* [M] float64 preconditioner, plan order  */
  const double* eps;               /* HOST [d] l2 bounds                      */
  const float* x_true;             /* optional [ny][nx] reference for SNR     */
  const float* W;                  /* optional [9][ny][nx] re-weights (Algorithm 1),
                                      NULL = identity                          */
  int32_t prox;                    /* PPD_PROX_* (0 = Algorithm 2)            */
  int32_t n_newton;                /* Newton steps for PPD_PROX_EXACT (0 -> 12) */
  const uint8_t* block_active;     /* optional DEVICE [d] active set D of the
                                      iterations of this call (randomised
                                      Algorithm 3): block j's v_j and z_j
                                      are updated only where nonzero; NULL =
                                      all blocks; fused form only            */
  const uint8_t* basis_active;     /* optional DEVICE [9] active set P of SARA
                                      bases (0 = Dirac, p = db-p; randomised
                                      Algorithm 3); NULL = all bases         */
  int32_t persistent;              /* PPD_PERSIST_AUTO (0): with n_itr > 1
                                      in the fused form and Algorithm 2, the
                                      n_itr - 1 middle steps run as one
                                      persistent launch with the per-point
                                      state in registers and bounded waits
                                      for each block's partial norms, when
                                      the plan's points fit the device at
                                      once (about 1.5M visibilities) and no
                                      3072 consecutive plan-order points
                                      span more than 4 blocks (the launch
                                      runs beside the SARA branch of its
                                      iteration, whose launches never wait
                                      on it; work that other streams run
                                      beside it and that waits itself, such
                                      as another plan's persistent launch,
                                      can make a wait give up);
                                      PPD_PERSIST_OFF (1): one launch pair
                                      per step                               */
  int32_t spin_limit;              /* polls of one wait of the persistent
                                      launch before it gives up (0: 2^20);
                                      a give-up
                                      makes every workgroup finish and the
                                      next call that reads statistics return
                                      PPD_EDEVICE                            */
  int32_t stats_every;             /* > 0: the statistics of every
                                      stats_every-th iteration of the call are
                                      also reduced on the device while the
                                      iterations run (a stopping test's work,
                                      no host synchronisation), into
                                      stats_history if given; 0: only those of
                                      the last iteration, if stats / residual
                                      are requested                          */
  int32_t pad2_;
  double* stats_history;           /* optional DEVICE [n_iter / stats_every]
                                      [8 + d]: row k is iteration
                                      (k + 1) stats_every's rel_change, ||x||,
                                      SNR dB (NaN without x_true),
                                      max_j r_j / eps_j, four raw FP64 sums and
                                      r_j = ||Theta_j G_j F Z x~ - y_j||      */
} ppd_params;

typedef struct {
  int64_t iter;          /* state->iter after the call                       */
  double rel_change;     /* ||x_t - x_{t-1}|| / ||x_t|| of the last iteration */
  double x_norm;         /* ||x_t||                                          */
  double snr_db;         /* 20 log10(||x_true|| / ||x_true - x_t||), NaN if no x_true */
  double residual_max;   /* max_j ||Theta_j G_j F Z x~_{t-1} - y_j|| / eps_j  */
} ppd_stats;

/* Run n_iter iterations of Algorithm 3 on `state`.  Every block and basis
 * is updated each iteration unless params->block_active / basis_active name
 * active subsets (the randomised variant; the masks are read on the device
 * at each iteration, so the caller may rewrite them between calls).
 * The data-dual update is read as
 * vbar_j = U_j (w_j - prox^U_h(w_j)), w_j = U_j^{-1} v_j + Theta_j G_j a,
 * with the prox approximated by n_itr Algorithm 2 iterations warm-started
 * from state->z (PPD_PROX_FB), or computed as by ppd_prox_metric
 * (PPD_PROX_EXACT; state->z then holds the last prox).  W_i = params->W
 * (identity if NULL).  If stats (HOST) is
 * non-NULL the call synchronises and fills it (and residual[d], HOST, if
 * non-NULL) from FP64 reductions of the last iteration.  The statistics
 * partials are formed only in iterations whose statistics are reduced
 * (every stats_every-th and the last); with use_graph the plan keeps two
 * captured iterations, one forming them and one not, and replays each
 * where it applies. */
int ppd_iterate(ppd_plan* plan, ppd_state* state, const ppd_params* params, int n_iter,
                ppd_stats* stats, double* residual);

/* Algorithm 1 (Sec. 3.2): n_reweights + 1 solves of iters_per_solve
 * iterations of Algorithm 3 each (as ppd_iterate with params), every solve
 * warm-started from the state the previous one left.  The first solve uses
 * params->W (NULL = identity); after solve k < n_reweights the weight
 * parameter becomes omega^(k+1) = decay^(k+1) omega0 and the re-weights
 * W = omega / (omega + |Psi^H x|) of the state's image (as ppd_reweight)
 * are written into W_work, which the next solve uses.  W_work: DEVICE
 * [9][ny][nx] float32, caller-owned, required when n_reweights > 0 and
 * not aliasing params->W.  stats: optional HOST [n_reweights + 1], the
 * statistics of each solve's last iteration (the call then synchronises
 * after each solve); params->stats_history, if given, ends with the rows of
 * the last solve (each solve is one ppd_iterate call).  omega0 > 0,
 * 0 < decay; omega is passed to the re-weighting in float32 and must stay
 * > 0 there.  Returns the first error of a solve or a re-weighting (the
 * state then holds the iterate so far). */
int ppd_reweighted(ppd_plan* plan, ppd_state* state, const ppd_params* params, int n_reweights,
                   int iters_per_solve, double omega0, double decay, float* W_work, ppd_stats* stats);

/* ---- differentiable pieces of Algorithm 3 (unrolled iterations) ------- */
/* One iteration of Algorithm 3 is, in the library's data flow,
 *   g = Theta G F Z x~ (ppd_phi),   (v', z') = dual update (g, v, z),
 *   c = Psi^H x~ (ppd_sara),        u' = sparsity update (u, c),
 *   x' , x~' = primal update (x, Re Phi^H v' (ppd_phit), Psi u' (ppd_sara)).
 * Each update below has a vector-Jacobian product (VJP): given the
 * gradients of a real loss with respect to its outputs, the gradients with
 * respect to its inputs, in torch's convention for complex arrays
 * (dL/dRe + i dL/dIm).  U, eps, alpha and the step sizes are constants.
 * All arrays are DEVICE arrays of the plan's sizes; no output may alias an
 * input.  Asynchronous on the plan's stream. */

/* Data-dual update (the generalised Moreau step of Algorithm 3 with
 * Algorithm 2 for the prox, Sec. 4.1), per block j of plan-order points:
 * w = U^-1 v + g, z_0 = z, z_s = P_B(z_{s-1} - mu U (z_{s-1} - w)) for
 * s = 1..n_itr, v' = v + lambda (U (w - z_n) - v), z' = z_n.  g, y, v,
 * v_out: [M] complex64; U: [M] float64; z, z_out: [M] complex128; eps: HOST
 * [d].  zs: optional [n_itr][M] complex128 receiving z_1..z_n (needed by the
 * VJP); FP64 arithmetic and block norms. */
int ppd_dual_update(ppd_plan* plan, const float* g, const float* y, const double* U, const double* eps,
                    const float* v, const double* z, int n_itr, double mu, double lambda, float* v_out,
                    double* z_out, double* zs);
/* VJP of ppd_dual_update (same inputs and the zs it wrote): from gv_out
 * ([M] complex64, NULL = 0) and gz_out ([M] complex128, NULL = 0), the
 * gradients g_g, g_v, g_y ([M] complex64, each optional) and g_z ([M]
 * complex128, required).  Through P_B the Jacobian is the identity inside
 * the ball and (eps / r)(I - d d^T / r^2) outside (d = q - y, r = ||d||),
 * applied with a block inner product per step. */
int ppd_dual_update_vjp(ppd_plan* plan, const float* g, const float* y, const double* U, const double* eps,
                        const float* v, const double* z, int n_itr, double mu, double lambda, const double* zs,
                        const float* gv_out, const double* gz_out, float* g_g, float* g_v, double* g_z,
                        float* g_y);
/* Sparsity dual update per coefficient ([9][ny][nx] float32):
 * u' = u + lambda (clip(u + c, +-alpha) - u), the clip being (I - S_alpha) of
 * Sec. 3.3.  VJP: g_u = (1 - lambda + lambda m) g_out, g_c = lambda m g_out,
 * m = [|u + c| < alpha] (g_u, g_c optional). */
int ppd_sparsity_update(ppd_plan* plan, const float* u, const float* c, float alpha, float lambda, float* u_out);
int ppd_sparsity_update_vjp(ppd_plan* plan, const float* u, const float* c, float alpha, float lambda,
                            const float* g_out, float* g_u, float* g_c);
/* Primal update per pixel ([ny][nx] float32; FP64 arithmetic):
 * xbar = P_C(x - tau (eta a + zeta b)), x' = x + lambda (xbar - x),
 * x~' = 2 xbar - x, with a = Re Phi^H v' and b = Psi u'.  VJP from gx_out,
 * gxt_out (NULL = 0): with m = [x - tau (eta a + zeta b) > 0] and
 * gbar = m (lambda gx_out + 2 gxt_out), g_x = (1 - lambda) gx_out - gxt_out
 * + gbar, g_a = -tau eta gbar, g_b = -tau zeta gbar (each optional). */
int ppd_primal_update(ppd_plan* plan, const float* x, const float* a, const float* b, double tau, double eta,
                      double zeta, double lambda, float* x_out, float* xt_out);
int ppd_primal_update_vjp(ppd_plan* plan, const float* x, const float* a, const float* b, double tau, double eta,
                          double zeta, double lambda, const float* gx_out, const float* gxt_out, float* g_x,
                          float* g_a, float* g_b);

/* ---- per-kernel timing (HIP events around each launch) ----------------- */
/* When enabled, the plan records a pair of HIP events around every kernel
 * it launches (not inside captured graphs).  ppd_timing_read synchronises
 * and returns, for up to `cap` kernel kinds, the name, launch count and
 * total milliseconds since the last reset. */
int ppd_timing_enable(ppd_plan* plan, int on);
int ppd_timing_reset(ppd_plan* plan);
int ppd_timing_read(ppd_plan* plan, int cap, const char** names /* HOST */,
                    int64_t* counts /* HOST */, double* total_ms /* HOST */, int* n_kinds);

/* ---- host-side helpers (no device work; used by CPU tests) ------------- */
/* The 8 per-axis Kaiser-Bessel interpolation weights the kernels use, for
 * n fractional offsets s in [0, 1): w[i][m] ~ phi(s_i + 3 - m), m = 0..7,
 * evaluated exactly as on the device (degree-9 polynomial per tap, float32
 * Horner).  HOST pointers. */
int ppd_kb_weights_host(double kb_beta, int64_t n, const float* s, float* w);
/* Daubechies-p low-pass filter (p = 1..8, 2p taps) as the library computes
 * it (float64, before rounding to float32).  HOST pointer. */
int ppd_daubechies_host(int p, double* h);

#ifdef __cplusplus
}
#endif
#endif /* PPD_H */
