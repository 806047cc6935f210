/*
 * gllmg — matrix-free high-order continuous-FE multigrid on AMD MI355X (gfx950).
 *
 * The method is the one compared by Sundar, Stadler and Biros, "Comparison of Multigrid
 * Algorithms for High-order Continuous Finite Element Discretizations": the Poisson problem
 * -div(mu grad u) = f with u = 0 on the boundary (§2, Eq. (Poisson)), discretized with
 * tensorized GLL nodal bases of order p <= 16 on a structured quad/hex mesh of the image of
 * the unit square/cube under a smooth map (§2.3), solved with h- or p-multigrid V-cycles
 * (§3.1) using Jacobi or Chebyshev-accelerated Jacobi smoothing (§3.2), as a solver or as
 * the preconditioner of CG (Algorithm 1). The operator is never assembled: every product
 * with A runs as a sum-factorized element kernel (§2.3, the O(p^4) tensorized matvec).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a gllmg_status; no C++ exception crosses this interface. On any
 *   status other than GLLMG_OK, gllmg_last_error() returns a message (thread-local, valid
 *   until the next call on the same thread). On error, outputs are left untouched except
 *   where a function says otherwise (GLLMG_ENOTCONV).
 * - Vectors are DEVICE pointers owned by the caller (for example the data pointer of a
 *   contiguous torch tensor), of the precision named by the gllmg_prec argument: double for
 *   GLLMG_F64, float for GLLMG_F32. A level vector has nnodes entries (gllmg_level_info):
 *   the nodes of the (n_x p + 1) x (n_y p + 1) [x (n_z p + 1)] grid, lexicographic with x
 *   fastest, g = i_x + N_x (i_y + N_y i_z). Entries at boundary nodes are ignored on input
 *   (treated as 0) and written as 0 on output (homogeneous Dirichlet data).
 * - Pointers must be aligned to their element size; input and output vectors must not alias
 *   unless a function says so.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream). All device work
 *   of a call is enqueued on it. Functions marked "asynchronous" return without waiting;
 *   the others synchronize the stream before returning.
 * - Levels are numbered 0 (finest) to nlevels-1 (coarsest).
 * - A problem is not reentrant: calls on one problem must not overlap. Distinct problems may
 *   be used concurrently from different threads on different streams.
 */
#ifndef GLLMG_H
#define GLLMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GLLMG_OK = 0,
  GLLMG_EINVAL = 1,       /* invalid argument, field or map (mu <= 0, detJ <= 0, ...)      */
  GLLMG_ENOMEM = 2,       /* workspace too small, or device allocation failed              */
  GLLMG_EDEVICE = 3,      /* a HIP runtime call failed                                     */
  GLLMG_ENOTCONV = 4,     /* a solve reached maxit; x holds the last iterate, stats filled */
  GLLMG_EBREAKDOWN = 5,   /* NaN/Inf residual or a non-positive curvature p^T A p          */
  GLLMG_EUNSUPPORTED = 6  /* the request needs data the problem was not set up with        */
} gllmg_status;

typedef enum { GLLMG_F64 = 0, GLLMG_F32 = 1 } gllmg_prec;

/* Hierarchies (§3.1): H keeps p and halves the elements per axis; P takes p -> ceil(p/2) down to
 * 1, then halves the elements; LOW (§3.1.3, a first-order operator whose cells have the order-p
 * nodes as vertices) keeps the order-p level, then a level of first-order cells
 * whose vertices are exactly the order-p nodes (n_e p cells per axis, same node numbering), then
 * halves that first-order grid (each coarser level on every other node). With LOW the solvers'
 * preconditioner is low_cycles sweeps x <- x + V_1 (r - A_1 x) from x = 0 of the first-order
 * operator A_1 and its V-cycle V_1 (levels 1 and below): an approximation of A_1^{-1} that tends
 * to it as the sweeps grow (the paper applies A_1^{-1} exactly). GLL quadrature only. */
enum { GLLMG_HIER_H = 0, GLLMG_HIER_P = 1, GLLMG_HIER_LOW = 2 };
/* Coarsening rule: halving the elements goes on while every axis has an even count and the
 * halved level keeps an interior node. With coarse_unknowns = k > 0 it also stops at the first
 * first-order level (p = 1, reached by any of the hierarchies) that has at most k interior
 * unknowns: that level is the coarsest and is solved exactly (§3, the coarse-grid direct solve;
 * on the GPU one exact solve of a few thousand unknowns costs less than the V-cycle launches of
 * the levels below it). max_levels then truncates the plan. */
/* Smoothers (§3.2, §4.3, §4.4.3):
 *   JACOBI        nu sweeps x += omega D^{-1} (b - A x)                    (paper: omega = 2/3)
 *   CHEBYSHEV     one degree-nu Chebyshev polynomial in D^{-1} A on [cheb_lo lambda, lambda]
 *   SSOR          nu symmetric Gauss-Seidel steps (a forward and a backward sweep each) in a
 *                 multicolor order of n^2 colors, n = p + 1: node (gx, gy[, gz]) has color
 *                 (gx mod n) + n (gy mod n) in 2D, ((gx + gz) mod n) + n ((gy + gz) mod n) in 3D;
 *                 colors 0..n^2-1 forward, then back; relaxation omega (paper: 1, SSOR(2,1))
 *   L1_JACOBI     nu sweeps x += omega D_l1^{-1} (b - A x), (D_l1)_ii = sum_j |A_ij| over the
 *                 interior row (paper: omega = 2/3)
 *   BLOCK_JACOBI  nu sweeps x += omega B^{-1} (b - A x), B = A restricted to the blocks of
 *                 element-owned interior nodes (along each axis an element owns its local
 *                 nodes 0..p-1, the last element also p), inverted exactly at setup
 *                 (paper: omega = 2/3). */
enum { GLLMG_SMOOTH_JACOBI = 0, GLLMG_SMOOTH_CHEBYSHEV = 1, GLLMG_SMOOTH_SSOR = 2,
       GLLMG_SMOOTH_L1_JACOBI = 3, GLLMG_SMOOTH_BLOCK_JACOBI = 4 };
enum { GLLMG_MODE_PCG = 0, GLLMG_MODE_MG = 1, GLLMG_MODE_IR = 2 };
/* Quadrature (§2.3): GLL collocation (the nodes are the (p+1)^d quadrature points: diagonal mass,
 * the stiffness couples a node with the coordinate planes through it) or the paper's Gauss rule
 * with p+1 Gauss-Legendre points per axis (geometry and mu at the Gauss points, dense element
 * matrices, consistent mass in gllmg_rhs). The Gauss rule takes the Jacobi and Chebyshev
 * smoothers (the SSOR coloring and the l1/block entries are built for collocation). */
enum { GLLMG_QUAD_GLL = 0, GLLMG_QUAD_GAUSS = 1 };

/* Field families, evaluated on the device at every level's nodes (physical coordinates
 * x = Phi(X) for coefficients and right-hand sides, reference coordinates X for maps).
 *   MAP_IDENTITY      Phi(X) = X
 *   MAP_WARP_SINE     3D: Phi = (X + a sY sZ, Y + a sZ sX, Z + a sX sY), sW = sin(2 pi W);
 *                     2D: Phi = (X + a sY, Y + a sX);            param[0] = a
 *   MAP_AFFINE        Phi(X) = M X + c; param = M (d*d, row-major) then c (d)
 *   CONST             param[0]
 *   EXP_SINE_PRODUCT  exp(param[0] prod_i sin(2 pi (x_i + param[1+i])))
 *   EXP_FOURIER       exp(sqrt(2/J) sum_j a_j cos(2 pi k_j.x + phi_j)); nmodes = J and
 *                     modes = host array of J rows [k0, k1, k2, a, phi] (copied at setup)
 *   SIN_PRODUCT       param[0] prod_i sin(param[1] pi x_i)
 *   COS2_SUM          param[0] + param[1] sum_i cos^2(param[2] pi x_i)   (paper §4.1 form)
 *   MAP_CALLBACK      any map Phi given by the caller (the smooth diffeomorphism of §2.3):
 *                     fn(X, npts, dim, x, ctx) writes x = Phi(X) for npts reference points X
 *                     (row-major npts x dim in, npts x dim out)
 *   FIELD_CALLBACK    any coefficient mu(x) given by the caller (§2, Eq. (Poisson)):
 *                     fn(x, npts, dim, out, ctx) writes out[i] = mu(x_i) at npts physical points
 * Callbacks run only inside gllmg_setup, on the calling thread, once per level, with the points
 * of every node of that level in node order (collocated quadrature needs Phi and mu at the nodes
 * only); their values are copied to the device. After setup a problem with a callback map does
 * not provide gllmg_node_coords or gllmg_eval_field (EUNSUPPORTED), and gllmg_eval_field does not
 * take a callback field (EINVAL). */
enum {
  GLLMG_MAP_IDENTITY = 0, GLLMG_MAP_WARP_SINE = 1, GLLMG_MAP_AFFINE = 2, GLLMG_MAP_CALLBACK = 3,
  GLLMG_FIELD_CONST = 10, GLLMG_FIELD_EXP_SINE_PRODUCT = 11, GLLMG_FIELD_EXP_FOURIER = 12,
  GLLMG_FIELD_SIN_PRODUCT = 13, GLLMG_FIELD_COS2_SUM = 14, GLLMG_FIELD_CALLBACK = 20
};
#define GLLMG_MAX_MODES 64

typedef void (*gllmg_field_fn)(const double* pts, int64_t npts, int32_t dim, double* out,
                               void* ctx);

typedef struct {
  int32_t kind;
  int32_t nmodes;
  double param[12];
  const double* modes;   /* host pointer, nmodes x 5 doubles, or NULL */
  gllmg_field_fn fn;     /* MAP_CALLBACK / FIELD_CALLBACK: the host function, else NULL */
  void* ctx;             /* passed to fn unchanged */
} gllmg_field;

typedef struct {
  int32_t dim;            /* 2 or 3                                                        */
  int32_t nelem[3];       /* elements per axis (>= 1); nelem[2] ignored in 2D              */
  int32_t order;          /* polynomial order p, 1..16                                     */
  int32_t hierarchy;      /* GLLMG_HIER_H, GLLMG_HIER_P or GLLMG_HIER_LOW (see above)        */
  int32_t max_levels;     /* 0: as many levels as the rule allows; else keep the finest k  */
  int32_t smoother;       /* GLLMG_SMOOTH_*                                                */
  int32_t nu_pre;         /* sweeps / Chebyshev degree / SSOR steps before the correction   */
  int32_t nu_post;        /* ... and after it                                              */
  double omega;           /* Jacobi-type damping (paper 2/3) or SSOR relaxation (paper 1)  */
  double cheb_lo;         /* Chebyshev interval [cheb_lo * lambda, lambda] (paper: 1/4)    */
  double cheb_safety;     /* lambda = cheb_safety x the Ritz estimate                      */
  int32_t eig_steps;      /* Lanczos/Arnoldi steps for lambda_max (paper: 10)             */
  int32_t vcycle_prec;    /* GLLMG_F64, or GLLMG_F32 for the mixed-precision V-cycle        */
  uint64_t eig_seed;      /* seed of the SplitMix64 start vector                           */
  int32_t quadrature;     /* GLLMG_QUAD_GLL (default) or GLLMG_QUAD_GAUSS                  */
  int32_t low_cycles;     /* GLLMG_HIER_LOW: first-order V-cycle sweeps per preconditioning  */
  int32_t coarse_unknowns;/* 0, or k in [1, 4096]: see the coarsening rule above             */
  int32_t ir_inner;       /* 0, or k in [1, 100]: GLLMG_MODE_IR's FP32 CG steps per refinement */
} gllmg_config;

typedef struct gllmg_problem gllmg_problem;

typedef struct {
  int32_t iters;            /* V-cycles applied (= CG iterations in PCG mode)              */
  int32_t converged;
  double relres;            /* ||r_k|| / ||r_0|| of the iteration's own residual            */
  double relres_true;       /* ||b - A x|| / ||r_0|| recomputed at the end (FP64)          */
  double t_solve_s;         /* wall time from entry to return                              */
  int64_t applies[16];      /* operator products per level during the solve                */
  double* history;          /* optional caller array of maxit+1 residual norms (or NULL)   */
} gllmg_solve_stats;

/* Last error message of this thread. */
const char* gllmg_last_error(void);

/* Paper defaults: P-hierarchy, Chebyshev degree 4 pre/post, omega 2/3, [lambda/4, lambda],
 * 10 eigen steps, FP64 V-cycle. dim/nelem/order are left for the caller. */
void gllmg_config_default(gllmg_config* cfg);

/* Number of levels and device bytes a setup of cfg needs: the whole device footprint. After
 * gllmg_setup no call allocates device or pinned host memory, streams or events (they are all
 * made by gllmg_setup, so admission by this figure is exact); the only exception is the V-cycle
 * graph that gllmg_set_lmax and gllmg_set_graphs(1) capture again. */
gllmg_status gllmg_plan(const gllmg_config* cfg, int32_t* nlevels, size_t* device_bytes);

/* Build the hierarchy: per level the geometric factors G = w mu detJ J^{-1} J^{-T} at every
 * GLL point (§2.3), the operator diagonal (§3.2.1), lambda_max of D^{-1} A (§3.2.2), the
 * transfer tables (§2.2) and, on the coarsest level, the dense inverse for the exact coarse
 * solve (only if that level has at most 4096 interior unknowns; otherwise the problem still
 * supports products and smoothing, and gllmg_vcycle / gllmg_solve return EUNSUPPORTED). device_ws / ws_bytes: caller memory of at least gllmg_plan's size, kept until
 * gllmg_destroy (or NULL / 0: the library allocates it). Synchronous.
 * Errors: EINVAL for bad sizes, mu <= 0 or non-finite at a node, detJ <= 0 at a point;
 * ENOMEM if ws_bytes is too small. */
gllmg_status gllmg_setup(const gllmg_config* cfg, const gllmg_field* map, const gllmg_field* mu,
                         void* device_ws, size_t ws_bytes, void* stream, gllmg_problem** out);

gllmg_status gllmg_destroy(gllmg_problem* prob);

gllmg_status gllmg_num_levels(const gllmg_problem* prob, int32_t* nlevels);

/* Sizes and the Chebyshev bound of one level. Any output pointer may be NULL. */
gllmg_status gllmg_level_info(const gllmg_problem* prob, int32_t level, int64_t* nnodes,
                              int64_t* ninterior, int32_t* order, int32_t nelem[3],
                              double* lmax);

/* Replace a level's lambda_max (for example to use an externally computed bound). The level's
 * Chebyshev coefficients are recomputed and the solve's V-cycle graph is captured again here
 * (synchronously), so that the next solve replays it. */
gllmg_status gllmg_set_lmax(gllmg_problem* prob, int32_t level, double lmax);

/* Replay the solve's V-cycle from a HIP graph captured on first use (enable = 1, the
 * default) or launch its kernels one by one (enable = 0). Both execute the same kernels in
 * the same order and give bitwise identical results; the graph removes host launch gaps.
 * The graph is captured at setup, again by gllmg_set_lmax, and by this call if enable = 1 and
 * none exists. */
gllmg_status gllmg_set_graphs(gllmg_problem* prob, int32_t enable);

/* Whether gllmg_batch_solve may solve this problem with the persistent solver or in a launch
 * group (enable = 1, the default) or must give it its own stream (0). See gllmg_batch_solve. */
gllmg_status gllmg_set_persistent(gllmg_problem* prob, int32_t enable);

/* Physical node coordinates x = Phi(X) of a level: out[g * dim + a]. FP64. Asynchronous. */
gllmg_status gllmg_node_coords(const gllmg_problem* prob, int32_t level, double* out, void* stream);

/* A field at a level's physical node coordinates (all nodes). FP64. Asynchronous. */
gllmg_status gllmg_eval_field(const gllmg_problem* prob, int32_t level, const gllmg_field* f,
                              double* out, void* stream);

/* Load vector on the finest level: b_j = (f_h, phi_j) for the nodal interpolant f_h of f (§2.1):
 * under GLL quadrature (lumped mass)_j f_j, under Gauss quadrature the consistent mass times f;
 * 0 on the boundary. f_nodal (every node, boundary included), b: FP64. Asynchronous. */
gllmg_status gllmg_rhs(const gllmg_problem* prob, const double* f_nodal, double* b, void* stream);

/* diag(A_level) at interior nodes, 0 on the boundary (§3.2.1). Asynchronous. */
gllmg_status gllmg_diag(const gllmg_problem* prob, int32_t level, gllmg_prec prec, void* d,
                        void* stream);

/* y = A_level x (§2.3 matrix-free product). neumann = 1 skips the boundary condition on both
 * input and output (the full stiffness, whose null space holds the constants). x and y must
 * not alias. GLLMG_F32 needs a problem set up with vcycle_prec = GLLMG_F32. Asynchronous. */
gllmg_status gllmg_apply(const gllmg_problem* prob, int32_t level, gllmg_prec prec, int32_t neumann,
                         const void* x, void* y, void* stream);

/* The product of gllmg_apply for callers that cannot allocate device memory at any point of
 * their run (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation). Same arguments, kernels and results (bit for bit) as gllmg_apply; the element
 * vectors that the two-kernel product passes from its element pass to its node-order sum are
 * kept in a static device array of the library (32 MiB per device, 33,554,432 bytes, present
 * from the moment the library is loaded on a device) instead of the problem's workspace.
 * Limit: E * (p+1)^d * sizeof(element) <= 33,554,432 bytes on the level (for example 16^3
 * hexes at p = 8 or 8^3 at p = 16 in FP64); a larger level returns EINVAL and enqueues nothing.
 * Every call on one device shares that device's array: calls that overlap in time on one
 * device (different streams, different problems or threads) race and give wrong results, so
 * the caller orders them (one stream, or events). The array keeps the last call's contents;
 * nothing in it needs to start at zero. Asynchronous. */
gllmg_status gllmg_apply_noalloc(const gllmg_problem* prob, int32_t level, gllmg_prec prec,
                                 int32_t neumann, const void* x, void* y, void* stream);

/* `steps` Jacobi sweeps (omega) or one Chebyshev polynomial of degree `steps` on
 * [cheb_lo lambda, lambda] of D^{-1} A (§3.2), updating x in place. zero_guess = 1 treats x as
 * 0 on entry (one product fewer). Uses the level's internal scratch. Asynchronous. */
gllmg_status gllmg_smooth(const gllmg_problem* prob, int32_t level, gllmg_prec prec, const void* b,
                          void* x, int32_t steps, int32_t zero_guess, void* stream);

/* xf = P xc from level fine_level+1 to fine_level: P_ij = phi_j^{coarse}(p_i), the coarse
 * basis at the fine nodes in reference coordinates (§2.2, Eq. (Pstencil)). Asynchronous. */
gllmg_status gllmg_prolong(const gllmg_problem* prob, int32_t fine_level, gllmg_prec prec,
                           const void* xc, void* xf, void* stream);

/* rc = P^T rf (the restriction, §2.2). Asynchronous. */
gllmg_status gllmg_restrict(const gllmg_problem* prob, int32_t fine_level, gllmg_prec prec,
                            const void* rf, void* rc, void* stream);

/* e = V r: one V-cycle on the finest level with zero initial guess (§3, §4.3): nu_pre
 * smoothing steps, residual, restriction, recursive coarse correction (exact solve on the
 * coarsest level), prolongation, nu_post smoothing steps. prec selects the V-cycle
 * precision (GLLMG_F32 for a problem set up with vcycle_prec = GLLMG_F32). Asynchronous. */
gllmg_status gllmg_vcycle(const gllmg_problem* prob, gllmg_prec prec, const void* r, void* e,
                          void* stream);

/* Solve A x = b on the finest level. mode GLLMG_MODE_PCG: CG preconditioned by one V-cycle
 * per iteration (Algorithm 1); GLLMG_MODE_MG: x += V (b - A x). The V-cycle runs in the
 * problem's vcycle_prec; the outer iteration, residuals and dot products are FP64. Stops
 * when ||r|| <= rtol ||r_0|| (§4.3). b, x: FP64 device vectors; x is the initial guess on
 * entry. stats may be NULL. Synchronous. ENOTCONV: maxit reached (x = last iterate, stats
 * filled). EBREAKDOWN: non-finite residual or p^T A p <= 0. EUNSUPPORTED: the coarsest level
 * has more than 4096 interior nodes, so no exact coarse solve was set up.
 * GLLMG_MODE_IR (problems set up with vcycle_prec = GLLMG_F32 and ir_inner = k > 0): iterative
 * refinement. Each step forms r = b - A x in FP64, scales it by a power of two to norm about 1,
 * runs m steps of CG in FP32 on A e = r from e = 0 (FP32 products, FP32 V-cycle as the
 * preconditioner, FP32 vector updates, FP64 dot products), and adds e, scaled back, to x in
 * FP64; it stops when the FP64 residual meets rtol. m = k in the first step; later, the
 * smallest count that the previous step's mean reduction per CG step predicts to reach rtol,
 * at most k (a step that falls short is followed by another). stats: iters counts the inner CG steps (one
 * V-cycle each; maxit bounds them), history holds ||b - A x|| before the first and after every
 * refinement step, followed by -1 where the array has room,
 * relres = relres_true. gllmg_solve only (solve_begin and batch solves: EUNSUPPORTED). */
gllmg_status gllmg_solve(const gllmg_problem* prob, int32_t mode, const double* b, double* x,
                         double rtol, int32_t maxit, gllmg_solve_stats* stats, void* stream);

/* The same solve split into non-blocking steps, so that one host thread can drive many
 * problems on different streams and interleave them iteration by iteration (continuous
 * batching). gllmg_solve_begin enqueues r = b - A x and its norm on `stream` and returns.
 * gllmg_solve_poll never blocks: it consumes the iteration scalars that have arrived, enqueues
 * the next iteration and sets *done = 1 once the solve (including the final true residual) has
 * finished. gllmg_solve_end waits for completion if needed, fills stats and returns the status
 * gllmg_solve would have returned. Iterates and counts are identical to gllmg_solve. One solve
 * per problem at a time; b and x must stay valid until gllmg_solve_end. An error returned by
 * gllmg_solve_poll ends the solve (the stream is drained first; gllmg_solve_end is not called
 * afterwards) and the problem accepts a new gllmg_solve_begin. */
gllmg_status gllmg_solve_begin(gllmg_problem* prob, int32_t mode, const double* b, double* x,
                               double rtol, int32_t maxit, void* stream);
gllmg_status gllmg_solve_poll(gllmg_problem* prob, int32_t* done);
gllmg_status gllmg_solve_end(gllmg_problem* prob, gllmg_solve_stats* stats);

/* Device copy of `bytes` bytes (a multiple of 16; src and dst 16-byte aligned, not overlapping)
 * by a plain streaming kernel, 16 bytes per lane: the library's achievable-bandwidth reference
 * for its roofline figures. Asynchronous. */
gllmg_status gllmg_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Solve `count` independent problems (any mix of dimension, mesh, order and precision), all
 * ordered after `stream`; the call returns when every solve has finished. Three paths:
 * - In PCG mode, two or more problems that share one shape (dimension, elements, order,
 *   hierarchy, smoother, degrees and V-cycle precision; coefficients and maps may differ) form a
 *   launch group: one lockstep PCG in which every kernel is launched once for all of them, each
 *   problem leaving the launches when its own solve ends; each result equals gllmg_solve's bit
 *   for bit. A group copies b and x through level-0 workspace vectors that its solve does not
 *   use otherwise, keeps its per-problem offsets, flags and scalars in the first problem's
 *   workspace (at most 256 problems per group; more of one shape form several groups), and runs
 *   on the first problem's internal stream, driven by a host thread of its own (groups run
 *   concurrently with each other and with the other paths). Nothing is allocated by the call.
 * - Small problems without a same-shape partner (3D, FP32 V-cycle, at most 10,000 fine-level
 *   nodes and 16 levels, an exact coarse solve, maxit < 1024) are solved by one persistent
 *   kernel launch per finest order on `stream`, one workgroup per problem, each stopping on its
 *   own: the same steps, smoothers and transfers as gllmg_solve, with the workgroup's dot
 *   products summed in another fixed order (iterates agree to rounding, not bitwise).
 * - The remaining problems run on their own internal streams, advanced iteration by iteration
 *   from the host thread.
 * gllmg_set_persistent(prob, 0) sends a problem to its own stream. stats and status may be
 * NULL, else arrays of `count`. Every handle must be non-NULL and appear once (checked before
 * any solve starts: EINVAL). Returns GLLMG_OK if every solve converged, else the first error
 * other than ENOTCONV if any, else ENOTCONV (status[i] holds each problem's own status; a
 * problem that fails does not stop the others). */
gllmg_status gllmg_batch_solve(gllmg_problem* const* probs, const double* const* b,
                               double* const* x, int32_t count, int32_t mode, double rtol,
                               int32_t maxit, gllmg_solve_stats* stats, gllmg_status* status,
                               void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GLLMG_H */
