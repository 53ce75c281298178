/*
 * labfm.h -- C ABI of the MI355X (gfx950) LABFM library (liblabfm.so).
 *
 * Local Anisotropic Basis Function Method, King, Lind & Nasar,
 * arXiv:1912.06441.  The library covers the data-parallel hot path:
 *   1. neighbour sets of every node (Sec. 2: all j within radius 2h),
 *   2. per-node weights (Sec. 3.1: M_i = sum_j X_ji (x) W_ji, M_i Psi^d = C^d,
 *      w^d_ji = W_ji . Psi^d),
 *   3. operator application (Sec. 2 eq. general_do: L^d_i(u) = sum_j (u_j - u_i) w^d_ji),
 *   4. explicit RK4 time stepping with those operators (Sec. 5.1), and the
 *      viscous Burgers' equation on a velocity field (Sec. 5.3).
 *
 * Conventions shared by every entry point:
 *   - Pointers named as device pointers must point to memory on the
 *     context's device (hipMalloc, or torch tensors on that device); host
 *     structs are read during the call only.  The caller owns all memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call only enqueues work on `stream` and returns, except where
 *     a call says it synchronises.
 *   - Argument errors return LABFM_EINVAL before anything is enqueued and
 *     set a thread-local message readable with labfm_last_error().
 *   - Inputs are never modified, except R when neighbour growth is on.
 *   - Node order is the caller's; sorting nodes by space-filling curve
 *     before the calls gives coalesced gathers.
 *   - Positions and radii are FP64; indices are int32 (col) / int64 (row_ptr).
 */
#ifndef LABFM_H
#define LABFM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LABFM_OK = 0,
    LABFM_EINVAL = -1,      /* bad argument (see labfm_last_error)          */
    LABFM_ENOMEM = -2,      /* library scratch allocation failed            */
    LABFM_EHIP = -3,        /* a HIP runtime call failed                    */
    LABFM_EUNSUPPORTED = -4 /* valid request the library does not implement */
} labfm_err;

/* ABF family.  HERMITE: W_m(d) = H_a(sigma d_x) H_b(sigma d_y) phi(|d|)
 * (physicists' Hermite polynomials times a radial function).  PAPER:
 * W_m = d^a_x d^b_y W0(|d|) (Sec. 3.2), keeping only the dW0/dr term for
 * elements of total order >= 4 (App. A).  PAPER_D1: every element keeps only
 * the dW0/dr term, W_m = dW0/dr(|d|) d^a_x d^b_y |d| (the App. A truncation
 * applied to all elements; with this family the quadratic RBF shows the
 * stability limits of Table noise_limits and the Dirichlet rates of Table
 * heatss).  For the cone (dW0/dr constant) PAPER and PAPER_D1 coincide.
 * (a, b) follow the element order of the monomial vector X (Sec. 2 eq. 1). */
typedef enum { LABFM_ABF_HERMITE = 0, LABFM_ABF_PAPER = 1, LABFM_ABF_PAPER_D1 = 2 } labfm_abf;

/* Fundamental RBF (App. A): cone, quadratic, Wendland C6, Gaussian, and the
 * 2-D Wendland C2 (1 - q/2)^4 (1 + 2q).  Constants do not change weights. */
typedef enum {
    LABFM_RBF_WENDLAND_C2 = 0,
    LABFM_RBF_CONE = 1,
    LABFM_RBF_QUADRATIC = 2,
    LABFM_RBF_WENDLAND_C6 = 3,
    LABFM_RBF_GAUSSIAN = 4
} labfm_rbf;

/* Operators (bits; weight sets are written in increasing bit order).
 * Targets C^d (Sec. 2, Sec. 4.2): DX e1, DY e2, LAP e3 + e5,
 * BIHARM -(e10 + 2 e12 + e14) (i.e. -nabla^4, needs k >= 4),
 * TRIHARM e21 + 3 e23 + 3 e25 + e27 (nabla^6, needs k >= 6). */
enum {
    LABFM_OP_DX = 1,
    LABFM_OP_DY = 2,
    LABFM_OP_LAP = 4,
    LABFM_OP_BIHARM = 8,
    LABFM_OP_TRIHARM = 16,
    LABFM_OP_DZ = 32 /* three-dimensional calls only */
};

/* Precision of the weight computation.
 * FP64: basis, moment matrix, LU and refinement all in FP64.
 * MIXED: basis and moment matrix in FP32 on matrix cores (FP32 accumulate),
 *        FP32 LU, FP64 residual and FP64 weight refinement; nodes whose
 *        refinement does not converge are recomputed on the FP64 path.
 * MLP: as MIXED, but nodes of the network's order start the refinement from
 *        the network's Psi0 (labfm_wopts.mlp) instead of from a first solve
 *        with the FP32 factors.
 * MLP_NOLU: nodes of the network's order take w = W Psi0 as it stands, with
 *        no moment matrix and no factorisation; a node whose FP64 moment
 *        residual from Psi0 is at or below tol_pass is finished (iters 0),
 *        any other is solved by the FP64 LU path (iters 64 + its count).
 *        Other orders: as MIXED. */
typedef enum {
    LABFM_PREC_FP64 = 0,
    LABFM_PREC_MIXED = 1,
    LABFM_PREC_MLP = 2,
    LABFM_PREC_MLP_NOLU = 3
} labfm_prec;

/* Per-node status written by labfm_weights.  The weight calls are
 * asynchronous, so per-node numerical failures are reported here only: a call
 * returns LABFM_OK once its work is enqueued, whatever the nodes' statuses
 * turn out to be (no error code depends on per-node results, which would force
 * a synchronisation on every call). */
enum {
    LABFM_ST_OK = 0,             /* moment residual <= tol_pass              */
    LABFM_ST_NOT_CONVERGED = 1,  /* weights written, residual > tol_pass     */
    LABFM_ST_SINGULAR = 2,       /* zero/non-finite pivot; weights zero      */
    LABFM_ST_TOO_FEW = 3,        /* fewer neighbours than p; weights zero    */
    LABFM_ST_DEGENERATE = 4,     /* PAPER ABFs undefined (coincident node)   */
    LABFM_ST_ORDER_TOO_LOW = 5,  /* order cannot express a requested target  */
    LABFM_ST_TOO_MANY = 6        /* more than LABFM_MAX_NEIGHBOURS (2-D) or
                                    LABFM_MAX_NEIGHBOURS3 (3-D) neighbours:
                                    weights zero (an implementation limit of
                                    the weight kernels) */
};

#define LABFM_MAX_ORDER 8
#define LABFM_MAX_NEIGHBOURS 128
#define LABFM_MAX_ORDER3 6
#define LABFM_MAX_NEIGHBOURS3 256 /* 3-D orders 5 and 6 (p = 55, 83) need > 100 */

/* Axis-aligned domain; periodic axes use the minimum-image offset. */
typedef struct {
    double lo[2], hi[2];
    int periodic[2];
} labfm_domain;

/* Learned warm start (not part of the paper): a fully connected network from
 * stencil features (labfm_mlp_features, dims[0] = 3 kmax) to the ABF
 * coefficients Psi^d of eq. (lsys), dims[n_layers] = nops(ops) * p(order),
 * in operator-major order (Psi^d_m at index d p + m).  Hidden layers apply
 * SiLU, z * sigmoid(z); the last layer is linear, and with de-normalisation
 * its output y becomes Psi = mu + sd * y.  Products use BF16 operands with
 * FP32 accumulation; biases and activations are FP32.  All arrays are device
 * memory owned by the caller. */
#define LABFM_MLP_MAX_LAYERS 8
typedef struct {
    int n_layers;                         /* weight layers, 1..8                          */
    int dims[LABFM_MLP_MAX_LAYERS + 1];   /* widths, each 1..4096                         */
    const void* W[LABFM_MLP_MAX_LAYERS];  /* BF16 [dims[l+1]][dims[l]], row-major         */
    const float* b[LABFM_MLP_MAX_LAYERS]; /* FP32 [dims[l+1]]                             */
    const float* mu;                      /* FP32 [dims[n_layers]] output shift           */
    const float* sd;                      /* FP32 [dims[n_layers]] output scale           */
    int order;                            /* stencil order the network serves (1..8)      */
    unsigned ops;                         /* LABFM_OP_* bits of its output                */
    int kmax;                             /* neighbours per input, 1..128                 */
} labfm_mlp;

/* Gradient buffers (device FP32, layouts of W and b). */
typedef struct {
    float* W[LABFM_MLP_MAX_LAYERS];
    float* b[LABFM_MLP_MAX_LAYERS];
} labfm_mlp_grads;

/* Adam hyper-parameters (Kingma & Ba 2015). */
typedef struct {
    double lr, beta1, beta2, eps;
} labfm_adam;

typedef struct {
    int abf;           /* labfm_abf                                        */
    int rbf;           /* labfm_rbf                                        */
    double sigma;      /* Hermite argument scale (HERMITE family)          */
    unsigned ops;      /* LABFM_OP_* bits                                  */
    int prec;          /* labfm_prec                                       */
    double tol_stop;   /* refinement stops when ||C - X^T w||_inf <= this  */
    double tol_pass;   /* status OK when the final residual <= this        */
    int max_iters;     /* FP64 refinement updates at most, 0..63 (iters[] is
                          int8 and the MIXED path adds 64 for nodes it hands
                          to the FP64 path)                                */
    const labfm_mlp* mlp; /* network for LABFM_PREC_MLP (host struct), else NULL */
} labfm_wopts;

/* Message of the last failed call on this thread ("" if none). */
const char* labfm_last_error(void);

/* Context: device id, library scratch (bucket grid, work lists), stream-
 * independent.  One context per device; calls on one context must not
 * overlap in time (scratch is shared). */
labfm_err labfm_create(void** ctx, int device);
labfm_err labfm_destroy(void* ctx);

/* Neighbour sets (Sec. 2): row i lists every j != i with
 * (x_j - x_i)^2 + (y_j - y_i)^2 < R_i^2 (minimum image on periodic axes),
 * in ascending j.  Two phases:
 *   count pass (col == NULL): if grow != 0, R_i <- 1.1 R_i (at most
 *     max_grow times) while the count is below N_crit(order_i) =
 *     8, 21, 37, 57 for order <= 2, 4, 6, 8 (Sec. 3.2 critical stencil
 *     sizes); writes R (grown) and row_ptr[n+1]; synchronises `stream` and
 *     returns the total in *nnz_host.
 *   fill pass (col != NULL): writes col[row_ptr[n]] for the R and row_ptr
 *     of the count pass; asynchronous.
 * x, y, R: device FP64 [n]; order: device int8 [n] (used only when grow);
 * row_ptr: device int64 [n+1]; col: device int32 [nnz].
 * Nodes must lie in [lo, hi] on every axis. */
labfm_err labfm_build_neighbours(void* ctx, const double* x, const double* y, int64_t n,
                                 const labfm_domain* dom, double* R, const int8_t* order,
                                 int grow, int max_grow, int64_t* row_ptr, int32_t* col,
                                 int64_t* nnz_host, void* stream);

/* Weights (Sec. 3.1 eqs. w_abf, disc_form, lsys) for every node i with
 * order k_i (1..8), h_i = R_i / 2, scaled offsets d_j = r_ji / h_i:
 *   M = sum_j X(d_j) W(d_j)^T, M Psi = C^d, w_j = W(d_j) . Psi,
 * solved by row-then-column max equilibration and LU with partial
 * pivoting, refined on the weights (r = C - X^T w; w += W M^-1 r) in FP64,
 * and unscaled by h^l (l = 1, 1, 2, 4, 6 for DX, DY, LAP, BIHARM, TRIHARM).
 * With LABFM_PREC_MLP(_NOLU) the network must serve exactly opt->ops; its features
 * and outputs for every node are computed first (library scratch of
 * 4 n dims[n_layers] bytes plus a chunk of 65536 nodes' activations).
 * Outputs (device): w64 [nops][nnz] FP64 and/or w32 [nops][nnz] FP32 (either
 * may be NULL, not both); status int8 [n]; resid FP32 [n] (final
 * max-norm moment residual over the operators); iters int8 [n] (FP64
 * refinement updates; on the MIXED path at most 30, and 64 + the FP64
 * path's count for nodes the mixed path handed to the FP64 path).  Failed
 * nodes get zero weights.  Asynchronous.
 * The FP64 path (and the FP64 recomputation of the other paths) runs two
 * kernels per order, passing each node's factors through library scratch:
 * 18,129 bytes per node for min(n, 262144) nodes (4.75 GB from n = 262144
 * on), kept by the context for later calls. */
labfm_err labfm_weights(void* ctx, const double* x, const double* y, int64_t n,
                        const labfm_domain* dom, const double* R, const int8_t* order,
                        const int64_t* row_ptr, const int32_t* col, int64_t nnz,
                        const labfm_wopts* opt, double* w64, float* w32, int8_t* status,
                        float* resid, int8_t* iters, void* stream);

/* labfm_weights without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): the same computation and, bit for bit, the same results
 * as labfm_weights, for opt->prec LABFM_PREC_FP64 or LABFM_PREC_MIXED; its
 * FP64 work runs in one kernel per order, which keeps each node's factors on
 * chip instead of in labfm_weights' factor scratch
 * (LABFM_PREC_MLP returns LABFM_EUNSUPPORTED).  Its work lists live in a
 * fixed library array of (2 LABFM_NOALLOC_MAX_NODES + 40) int32 (about 8 MiB)
 * that every GPU the library runs on holds until the process ends; n above
 * LABFM_NOALLOC_MAX_NODES returns LABFM_EINVAL.  Every call on one GPU shares
 * that array (it keeps the last call's contents; what must start at zero is
 * cleared by a kernel inside the call), so calls that overlap in time on one
 * GPU race: issue them on one stream, or order them.  No kernel timing is
 * recorded.  Arguments, layouts and outputs as labfm_weights; asynchronous. */
#define LABFM_NOALLOC_MAX_NODES (1 << 20)
labfm_err labfm_weights_noalloc(void* ctx, const double* x, const double* y, int64_t n,
                                const labfm_domain* dom, const double* R, const int8_t* order,
                                const int64_t* row_ptr, const int32_t* col, int64_t nnz,
                                const labfm_wopts* opt, double* w64, float* w32, int8_t* status,
                                float* resid, int8_t* iters, void* stream);

/* Batched weights: nsets independent node sets, each with its own arrays,
 * domain and outputs (layouts as in labfm_weights; col holds indices within
 * the set).  One pair of persistent kernels per order (factor, then weights
 * and refinement, as in labfm_weights) covers the nodes of every set, so
 * small and low-order sets share the GPU instead of each filling it alone;
 * the batch keeps its own factor scratch (18,129 bytes per node for up to
 * 262144 nodes at a time), allocated before any graph capture.
 * prec FP64 or MIXED (LABFM_PREC_MLP returns LABFM_EUNSUPPORTED).
 * use_graph != 0: work lists, weight kernels and the FP64 fallback of the
 *   whole batch are captured once as a HIP graph per (sets, options, stream)
 *   and replayed by later calls with the same arguments (the graph owns its
 *   own work-list buffers; replays read the sets' current array contents).
 * Autotuning (MIXED): the first time an order is seen under (abf, rbf, ops),
 *   the mixed route (matrix-core assembly + FP32 LU + FP64 refinement, with its
 *   FP64 retries) and the FP64 route are timed on up to 4096 of its nodes and
 *   the faster one is used from then on; both routes meet the same residual
 *   gate.  The first call synchronises `stream` for this; later calls are
 *   asynchronous.  Total node count < 2^31. */
typedef struct {
    const double* x;
    const double* y;
    int64_t n;
    labfm_domain dom;
    const double* R;
    const int8_t* order;
    const int64_t* row_ptr;
    const int32_t* col;
    int64_t nnz;
    double* w64;
    float* w32;
    int8_t* status;
    float* resid;
    int8_t* iters;
} labfm_node_set;

labfm_err labfm_weights_batched(void* ctx, int nsets, const labfm_node_set* sets, const labfm_wopts* opt,
                                int use_graph, void* stream);

/* The autotuner's choice for `order` under (abf, rbf, ops): *route = 0 (not
 * tuned yet), 1 (mixed kernels) or 2 (FP64 kernels); sample times in ms and
 * the sample size (nodes), each may be NULL. */
labfm_err labfm_autotune_query(void* ctx, int abf, int rbf, unsigned ops, int order, int* route, double* ms_mixed,
                               double* ms_fp64, int64_t* sample);

/* out[s] = sum_k coef[k] * w64[k][s] for s < nnz (a linear combination of
 * weight sets is the weight set of the combined target, C^d being linear).
 * coef: host [nsets]; out64 and/or out32 device [nnz].  Asynchronous. */
labfm_err labfm_combine(void* ctx, const double* w64, int nsets, const double* coef,
                        int64_t nnz, double* out64, float* out32, void* stream);

/* Operator application (Sec. 2 eq. general_do), nops operators sharing one
 * neighbour structure: out[d][i] = sum_{s in row i} w[d][s] (u[col[s]] - u[i]).
 * dtype 0: w, u, out FP32; dtype 1: FP64.  w [nops][nnz], out [nops][n]
 * (device).  Asynchronous. */
labfm_err labfm_apply_operator(void* ctx, const int64_t* row_ptr, const int32_t* col, int64_t n,
                               int64_t nnz, int nops, const void* w, int dtype, const void* u,
                               void* out, void* stream);

/* Classical RK4 (Sec. 5.1) on du/dt = L_lin(u) - gamma B(B(u)), where L_lin
 * uses w_lin and B (optional) uses w_bh; with B the -nabla^4 stencil,
 * B o B approximates nabla^8 (composed hyperviscosity).  Dirichlet nodes
 * (Sec. 5.1, heat equation with prescribed boundary values): where fixed[i]
 * is non-zero every stage derivative of node i is zero, so u[i] keeps the
 * value the caller put there; the other nodes still read it through their
 * stencils. */
typedef struct {
    const int64_t* row_ptr; /* device int64 [n+1]                   */
    const int32_t* col;     /* device int32 [nnz]                   */
    int64_t n, nnz;
    int dtype;              /* 0: FP32 weights and state; 1: FP64   */
    const void* w_lin;      /* device [nnz]                         */
    const void* w_bh;       /* device [nnz] or NULL                 */
    double gamma;           /* coefficient of B(B(u))               */
    double dt;
    const int8_t* fixed;    /* device int8 [n] or NULL (no Dirichlet nodes) */
} labfm_step_plan;

/* Advance u (device [n], dtype of the plan) by nsteps RK4 steps.
 * scratch: device, at least 5 n elements of the plan's dtype.
 * use_graph != 0 captures one step as a HIP graph and replays it.
 * Asynchronous. */
labfm_err labfm_step(void* ctx, const labfm_step_plan* plan, void* u, void* scratch, int nsteps,
                     int use_graph, void* stream);

/* Viscous Burgers' equation (Sec. 5.3, eq. burgers) for the velocity (u, v)
 * with classical RK4 (Sec. 5.1):
 *   du/dt = -(u L^x(u) + v L^y(u)) + nu L^L(u) + L^hv(u),
 *   dv/dt = -(u L^x(v) + v L^y(v)) + nu L^L(v) + L^hv(v),
 * nu = 1/Re; L^hv is an optional hyperviscosity operator (Sec. 4.2, e.g.
 * -100 h^4 nabla^4 or 8 h^6 nabla^6) whose coefficient the caller has folded
 * into w_hv (labfm_combine).  Dirichlet nodes (fixed[i] != 0) keep their
 * values, as in labfm_step, or, when dfix is given, take at RK4 stage q the
 * derivatives dfix[q n + i] (u) and dfix[(4 + q) n + i] (v) in place of the
 * right-hand side: the time derivative of a prescribed solution, e.g. the
 * analytic travelling wave on the nodes outside the domain (Sec. 5.3).  The
 * caller rewrites dfix between steps (stage q of the step from t at
 * t + c_q dt, c = 0, 1/2, 1/2, 1); a captured step reads it at replay. */
typedef struct {
    const int64_t* row_ptr; /* device int64 [n+1]                   */
    const int32_t* col;     /* device int32 [nnz]                   */
    int64_t n, nnz;
    int dtype;              /* 0: FP32 weights and state; 1: FP64   */
    const void* w_x;        /* device [nnz]: d/dx weights           */
    const void* w_y;        /* device [nnz]: d/dy weights           */
    const void* w_lap;      /* device [nnz]: Laplacian weights      */
    const void* w_hv;       /* device [nnz] or NULL                 */
    double nu;              /* viscosity 1/Re                       */
    double dt;
    const int8_t* fixed;    /* device int8 [n] or NULL              */
    const void* dfix;       /* device [2][4][n] of the plan's dtype, or NULL;
                               needs fixed                           */
} labfm_burgers_plan;

/* Advance (u, v) (device [n] each, dtype of the plan) by nsteps RK4 steps.
 * scratch: device, at least 6 n elements of the plan's dtype, aligned to two
 * elements (8 bytes FP32, 16 bytes FP64; the stage states of u and v are kept
 * there as pairs), not aliasing u or v.  use_graph != 0 captures one step as a HIP graph (kept while plan,
 * buffers and stream are unchanged) and replays it.  Argument errors return
 * LABFM_EINVAL before any launch.  Asynchronous. */
labfm_err labfm_burgers_step(void* ctx, const labfm_burgers_plan* plan, void* u, void* v, void* scratch,
                             int nsteps, int use_graph, void* stream);

/* Global Laplacian solve (Sec. 5.2, eq. poisson_system): A^L Phi = F, where
 * row i of A^L applies node i's Laplacian weights in difference form
 * (A_ij = w_ij for j in row i, A_ii = -sum_j w_ij) and a node with
 * fixed[i] != 0 has an identity row (A_ii = 1, Phi_i = F_i: Dirichlet data).
 * Solver: BiCGStab with a Jacobi preconditioner applied on the right, FP64,
 * started from the Phi passed in; it stops when ||F - A Phi||_2 <= tol ||F||_2,
 * when the recurrence breaks down, or after max_iters iterations. */
typedef struct {
    const int64_t* row_ptr; /* device int64 [n+1]                            */
    const int32_t* col;     /* device int32 [nnz]                            */
    int64_t n, nnz;
    const double* w_lap;    /* device FP64 [nnz]: Laplacian weights          */
    const int8_t* fixed;    /* device int8 [n] or NULL: Dirichlet rows       */
    double tol;             /* relative residual target, > 0                 */
    int max_iters;          /* >= 0                                          */
    int check_every;        /* iterations between host reads of the residual */
    const int32_t* center;  /* device int32 [n], values in [0, n), or NULL: row i
                               takes its differences about node center[i]
                               (Neumann ghost rows, see labfm_neumann_rows);
                               NULL: about node i itself.  Not range-checked,
                               like col */
} labfm_poisson_plan;

/* Rows of the global system enlarged by Neumann ghost rows (Sec. 5.2, eq. neu):
 * every node b on a Neumann boundary has a ghost node (outside the boundary,
 * part of the node set and of the neighbour sets), whose row enforces the
 * boundary condition at b through b's discrete normal derivative,
 *   A_gj = n_x w^x_bj + n_y w^y_bj (j in b's stencil), A_gb = -sum_j A_gj,
 * with (n_x, n_y) the unit normal at b pointing into the domain; every other
 * node keeps its own row with its Laplacian weights.  Inputs: the neighbour
 * sets of every node (row_ptr int64 [n+1], col int32 [nnz]) and its FP64 d/dx,
 * d/dy and Laplacian weights (w_x, w_y, w_lap [nnz]); parent int32 [n]: the
 * boundary node of a ghost, -1 for every other node (a value outside [0, n)
 * counts as -1); nx, ny FP64 [n]: the inward normal, read at ghost rows.
 * Outputs, in two passes as labfm_build_neighbours: out_col == NULL fills
 * out_row_ptr [n+1] and *nnz_host (synchronises stream); then out_col int32,
 * out_w FP64 [nnz_out] and out_center int32 [n] (out_center[g] = b for a
 * ghost, out_center[i] = i otherwise) for labfm_poisson_plan.  The right-hand
 * side of a ghost row is the Neumann datum at b.  All arrays device memory;
 * asynchronous (fill pass). */
labfm_err labfm_neumann_rows(void* ctx, const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                             const double* w_x, const double* w_y, const double* w_lap, const int32_t* parent,
                             const double* nx, const double* ny, int64_t* out_row_ptr, int32_t* out_col,
                             double* out_w, int32_t* out_center, int64_t* nnz_host, void* stream);

/* Solve in place: phi (device FP64 [n]) holds the initial guess on entry and
 * the solution on exit; F (device FP64 [n]) is not modified.  scratch: device,
 * at least 8 n doubles.  On return (the call synchronises `stream`) *iters,
 * *rel_resid (||F - A Phi|| / ||F|| of the returned Phi) and *converged (1 if
 * the tolerance was met) are set (host pointers, each may be NULL).  A
 * non-converged solve still returns LABFM_OK; argument errors return
 * LABFM_EINVAL before any launch. */
labfm_err labfm_poisson_solve(void* ctx, const labfm_poisson_plan* plan, const double* F, double* phi,
                              void* scratch, int* iters, double* rel_resid, int* converged, void* stream);

/* Incompressible Navier-Stokes in vorticity-streamfunction form (Sec. 5.4):
 *   d omega/dt = -(u L^x(omega) + v L^y(omega)) + nu L^L(omega),
 *   L^L psi = -omega,  u = L^y(psi),  v = -L^x(psi),
 * classical RK4 (Sec. 5.1) in FP64; at every stage psi is re-solved with
 * labfm_poisson_solve's method (warm-started from the previous psi) with the
 * rows marked in psi_fixed held at psi = 0 (on a periodic domain one pinned
 * node fixes the free constant). */
typedef struct {
    const int64_t* row_ptr; /* device int64 [n+1]                                 */
    const int32_t* col;     /* device int32 [nnz]                                 */
    int64_t n, nnz;
    const double* w_x;      /* device FP64 [nnz]: d/dx weights                    */
    const double* w_y;      /* device FP64 [nnz]: d/dy weights                    */
    const double* w_lap;    /* device FP64 [nnz]: Laplacian weights               */
    const int8_t* psi_fixed;/* device int8 [n] or NULL: rows with psi = 0         */
    double nu;              /* 1 / Re                                             */
    double dt;
    double tol;             /* relative residual of every stream-function solve   */
    int max_iters;          /* per solve                                          */
    int check_every;        /* per solve, as in labfm_poisson_plan                */
} labfm_ns_plan;

/* Advance omega (device FP64 [n]) by nsteps RK4 steps; psi (device FP64 [n])
 * holds the initial guess of the first solve on entry and the stream function
 * of the last step's first stage on exit.  scratch: device, at least 14 n
 * doubles, aliasing neither omega nor psi.  Synchronises `stream` at every
 * solve.  *solver_iters receives the BiCGStab iterations summed over all
 * solves and *all_converged 1 if every solve met tol (host pointers, each may
 * be NULL).  Argument errors return LABFM_EINVAL before any launch. */
labfm_err labfm_ns_step(void* ctx, const labfm_ns_plan* plan, double* omega, double* psi, void* scratch, int nsteps,
                        int* solver_iters, int* all_converged, void* stream);

/* ---- three dimensions ----------------------------------------------------
 * Sec. 3.1 gives p in 3-D (3, 9, 19, 34, 55, 83 for k = 1..6).  Element m is (a, b, c)
 * over total order n = 1..k with a = n..0, then b = n-a..0, c = n-a-b;
 * X_m = x^a y^b z^c / (a! b! c!); ABFs of the HERMITE family only,
 * H_a(s x) H_b(s y) H_c(s z) phi(|d|).  Operators: LABFM_OP_DX, _DY, _DZ
 * (target e1, e2, e3) and _LAP (e4 + e7 + e9, needs k >= 2); weight sets are
 * written in increasing bit order (dx, dy, lap, dz). */
typedef struct {
    double lo[3], hi[3];
    int periodic[3];
} labfm_domain3;

/* 3-D neighbour sets: j != i with |r_j - r_i| < R[i] (squared distance summed
 * x, y, z in that order, explicitly rounded), minimum image on periodic axes,
 * ascending j; no radius growth.  Two passes as labfm_build_neighbours: col
 * NULL fills row_ptr [n+1] and *nnz_host (synchronises stream); then the
 * caller allocates col [nnz] and calls again to fill it.  x, y, z, R: device
 * FP64 [n], nodes inside [lo, hi). */
labfm_err labfm_build_neighbours3(void* ctx, const double* x, const double* y, const double* z, int64_t n,
                                  const labfm_domain3* dom, const double* R, int64_t* row_ptr, int32_t* col,
                                  int64_t* nnz_host, void* stream);

/* 3-D weights of order k (1..LABFM_MAX_ORDER3 = 6; p = 3, 9, 19, 34, 55, 83,
 * Sec. 3.1) for every node, FP64 (opt->prec must be
 * LABFM_PREC_FP64 and opt->abf LABFM_ABF_HERMITE, else LABFM_EUNSUPPORTED);
 * the refinement, status, residual and iteration outputs are those of
 * labfm_weights.  w64: device [nops][nnz]; status int8 [n]; resid FP32 [n]
 * and iters int8 [n] may be NULL.  Asynchronous.  Orders 1..4 pass each
 * node's factors through library scratch (8 P^2 + 60 P + 1 bytes per node,
 * 11,289 at k = 4, for min(n, 262144) nodes), kept by the context. */
labfm_err labfm_weights3(void* ctx, const double* x, const double* y, const double* z, int64_t n,
                         const labfm_domain3* dom, const double* R, int k, const int64_t* row_ptr,
                         const int32_t* col, int64_t nnz, const labfm_wopts* opt, double* w64, int8_t* status,
                         float* resid, int8_t* iters, void* stream);

/* ---- learned warm start: features, network, training --------------------
 * Features of every node i < n (Sec. 2 stencil, scaled offsets d = r_ji / h_i,
 * h_i = R_i / 2): the row's neighbours ranked by (d_x^2 + d_y^2, j), the
 * nearest kmax written as feat[i][3t..3t+2] = (d_x, d_y, 1), missing slots
 * (0, 0, 0); rows with more than LABFM_MAX_NEIGHBOURS entries get all zeros.
 * feat: device FP32 [n][3 kmax].  Asynchronous. */
labfm_err labfm_mlp_features(void* ctx, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                             const double* R, const int64_t* row_ptr, const int32_t* col, int kmax, float* feat,
                             void* stream);

/* Training data of the warm start, made on the GPU: for every node i < n (all
 * taken at order k, 1..8; x, y hold every node col refers to) with
 * h_i = R_i / 2, the moment matrix of eq.
 * (disc_form) in scaled offsets, M[i] = sum_j X(d_j) W(d_j)^T, FP32 [n][p][p]
 * (row = monomial) as assembled, and the coefficients Psi^d of eq. (lsys) for
 * opt->ops (the FP64 path's equilibration, partial-pivot LU and one solve, no
 * refinement), FP32 [n][nops p] operator-major, which labfm_mlp_moment_loss
 * and the network's output scaling take.  opt->abf, rbf, sigma, ops are used;
 * prec, tolerances and max_iters are not.  status int8 [n] as labfm_weights
 * (OK, SINGULAR, TOO_FEW, TOO_MANY, DEGENERATE, ORDER_TOO_LOW); nodes that
 * are not OK get zeros.  All arrays device memory.  Asynchronous. */
labfm_err labfm_moment_systems(void* ctx, const double* x, const double* y, int64_t n, const labfm_domain* dom,
                               const double* R, int k, const int64_t* row_ptr, const int32_t* col, int64_t nnz,
                               const labfm_wopts* opt, float* M, float* psi, int8_t* status, void* stream);

/* Forward pass of B rows: in FP32 [B][dims[0]] -> out FP32 [B][dims[n_layers]]
 * (de-normalised when denorm != 0).  cache (device FP32, NULL for inference):
 * receives, per hidden layer l, the pre-activations Z_l then the activations
 * H_l, each [B][dims[l+1]] (labfm_mlp_cache_floats gives the size); the
 * backward pass reads it.  Asynchronous. */
labfm_err labfm_mlp_forward(void* ctx, const labfm_mlp* net, const float* in, int64_t B, float* out, float* cache,
                            int denorm, void* stream);
int64_t labfm_mlp_cache_floats(const labfm_mlp* net, int64_t B);

/* Backward pass: given dLoss/d(out) (dout, FP32 [B][dims[n_layers]], the
 * output before de-normalisation) and the forward cache of the same in,
 * writes dLoss/dW_l and dLoss/db_l (overwritten, not accumulated).
 * Asynchronous. */
labfm_err labfm_mlp_backward(void* ctx, const labfm_mlp* net, const float* in, const float* cache, const float* dout,
                             int64_t B, const labfm_mlp_grads* grads, void* stream);

/* Moment-residual loss of eq. (lsys) for the network output y [B][nops p]:
 * Psi_s = mu + sd * y_s, loss[s] = sum_d |M_s Psi^d_s - C^d|^2 (FP64, [B]),
 * dy = d(mean_s loss[s]) / dy (FP32 [B][nops p]).  M: FP32 [B][p][p], row =
 * monomial (M = sum_j X(d_j) W(d_j)^T, eq. disc_form).  Asynchronous. */
labfm_err labfm_mlp_moment_loss(void* ctx, const float* y, const float* M, const float* mu, const float* sd,
                                int order, unsigned ops, int64_t B, float* dy, double* loss, void* stream);

/* One Adam step (step number t >= 1) on count FP32 parameters with their
 * moments m, v; param_bf16 (optional) receives the updated values in BF16.
 * Asynchronous. */
labfm_err labfm_mlp_adam(void* ctx, float* param, const float* grad, float* m, float* v, void* param_bf16,
                         int64_t count, const labfm_adam* hp, int64_t t, void* stream);

/* dst (BF16) = src (FP32, round to nearest even), count elements.  Asynchronous. */
labfm_err labfm_mlp_cast_bf16(void* ctx, const float* src, void* dst, int64_t count, void* stream);

/* Kernel timing for measurement: while enabled, HIP events are recorded on
 * the launch stream around each kernel the library launches (outside graph
 * capture).  labfm_timing_read waits for the recorded kernels whose name
 * contains `filter` (NULL: all), returns their count and summed duration in
 * milliseconds, and forgets them.  Kernel names: neigh_count, neigh_fill,
 * weights64f_k1..k8 and weights64r_k1..k8 (the two FP64 kernels of an
 * order), weights64_k1..k8 (the single FP64 kernel), weights32_k1..k8,
 * weights3d_k1..k6 (every 3-D kernel of an order), apply_f32, apply_f64, step_graph,
 * step_direct, burgers_graph, burgers_direct, poisson_setup,
 * poisson_iterations, mlp_features, mlp_forward,
 * mlp_backward, mlp_loss, mlp_adam,
 * weights_batch_graph. */
labfm_err labfm_timing_enable(void* ctx, int enable);
labfm_err labfm_timing_read(void* ctx, const char* filter, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* LABFM_H */
