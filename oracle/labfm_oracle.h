/*
 * labfm_oracle.h -- plain FP64 CPU oracle for the LABFM hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library (no headers, kernels, tables or helpers).
 *
 * Everything here follows King, Lind & Nasar, "High order difference schemes
 * using the Local Anisotropic Basis Function Method" (arXiv:1912.06441):
 *   Sec. 2 eqs. (1)-(2)          monomial vector X, derivative vector D
 *   Sec. 2 eq. (general_do)      L_i(u) = sum_j (u_j - u_i) w_ji
 *   Sec. 3.1 eqs. (w_abf), (disc_form), (lsys)   w = W.Psi, M = sum X (x) W, M Psi = C
 *   Sec. 3.2 eq. (conic_abs) and App. A          ABFs from a fundamental RBF
 *   Sec. 4.2 (stability)         hyperviscosity target vectors
 *   Sec. 5.1                     classical RK4
 *   Sec. 5.3                     viscous Burgers' equation (RK4)
 *   Sec. 3.1 (3-D p)             three-dimensional monomials, Hermite ABFs, weights
 * Readings where the paper is silent are listed at each function.
 */
#ifndef LABFM_ORACLE_H
#define LABFM_ORACLE_H
#include <stdint.h>

#define OR_MAXK 8
/* largest number of elements p: 44 for a 2-D scheme of order 8, 83 for a 3-D
 * scheme of order 6 (the highest 3-D order here) */
#define OR_MAXP 84
#define OR_MAXK3 6

/* ABF families: HERMITE = H_a(s dx) H_b(s dy) phi(|d|); PAPER = D^(a,b) W0(|d|)
 * with the App. A truncation (only the dW0/dr term for total order >= 4). */
enum { OR_ABF_HERMITE = 0, OR_ABF_PAPER = 1, OR_ABF_PAPER_D1 = 2 };
enum { OR_RBF_WENDLAND_C2 = 0, OR_RBF_CONE = 1, OR_RBF_QUADRATIC = 2,
       OR_RBF_WENDLAND_C6 = 3, OR_RBF_GAUSSIAN = 4 };
/* operator bits, in output order */
enum { OR_OP_DX = 1, OR_OP_DY = 2, OR_OP_LAP = 4, OR_OP_BIHARM = 8, OR_OP_TRIHARM = 16,
       OR_OP_DZ = 32 /* 3-D only */ };
/* per-node status */
enum { OR_ST_OK = 0, OR_ST_NOT_CONVERGED = 1, OR_ST_SINGULAR = 2, OR_ST_TOO_FEW = 3,
       OR_ST_DEGENERATE = 4, OR_ST_ORDER_TOO_LOW = 5, OR_ST_TOO_MANY = 6 };
/* Longest stencil row the weights accept (an implementation limit, not the
 * paper's: the method itself takes any number of neighbours).  Longer rows get
 * OR_ST_TOO_MANY and zero weights, as the HIP library documents for its
 * LABFM_MAX_NEIGHBOURS (2-D) and LABFM_MAX_NEIGHBOURS3 (3-D, where orders 5
 * and 6 need 55 and 83 elements and so well over 100 neighbours). */
#define OR_NMAX 128
#define OR_NMAX3 256

typedef struct {
    double lo[2], hi[2];
    int periodic[2];
} or_domain;

typedef struct {
    double lo[3], hi[3];
    int periodic[3];
} or_domain3;

typedef struct {
    int family;        /* OR_ABF_* */
    int rbf;           /* OR_RBF_* */
    double sigma;      /* Hermite argument scale (HERMITE family) */
    unsigned ops;      /* OR_OP_* bits */
    double tol_stop;   /* refinement stops when ||C - X^T w||_inf <= tol_stop */
    int max_iters;     /* maximum refinement updates */
} or_wopts;

int or_p_of_k(int k);
int or_ncrit(int k);
void or_index_table(int k, int* ea, int* eb);
void or_monomials(int k, double dx, double dy, double* X);
int or_abfs(int family, int rbf, double sigma, int k, double dx, double dy, double* W);
int or_rbf_derivs(int rbf, double q, double* f /* f, f', f'', f''' */);
void or_hermite(int nmax, double t, double* H);

int64_t or_neighbours_brute(int64_t n, const double* x, const double* y, const or_domain* dom,
                            double* R, const int8_t* order, int grow, int max_grow,
                            int64_t* row_ptr, int32_t* col);
int64_t or_neighbours_cells(int64_t n, const double* x, const double* y, const or_domain* dom,
                            double* R, const int8_t* order, int grow, int max_grow,
                            int64_t* row_ptr, int32_t* col);

int or_node_weights(int k, int N, const double* dxh, const double* dyh, const or_wopts* o,
                    double* what /* [nops][N] scaled weights */, double* resid, int* iters,
                    double* Mhat /* optional p*p (row = monomial) */, double* cond1 /* optional */);
int or_targets(unsigned ops, int k, double* C /* [nops][p] */);
void or_stencils_psi(int64_t n, int k, int Nmax, const int32_t* N, const double* dxh, const double* dyh,
                     const or_wopts* o, double* psi /* [n][nops][p] */, int8_t* status, double* resid,
                     double* Mhat /* optional [n][p][p] */);
int or_weights(int64_t n, const double* x, const double* y, const or_domain* dom, const double* R,
               const int8_t* order, const int64_t* row_ptr, const int32_t* col, const or_wopts* o,
               double* w /* [nops][nnz] */, int8_t* status, double* resid, int8_t* iters);

void or_apply(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* w,
              const double* u, double* out);
void or_combine(int64_t nnz, int nsets, const double* w, const double* coef, double* out);
void or_rk4(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* w_lin,
            const double* w_bh, double gamma, double dt, int nsteps, double* u,
            const int8_t* fixed /* optional [n]: Dirichlet nodes, not advanced */);
void or_burgers_rk4(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* wx,
                    const double* wy, const double* wl, const double* whv /* or NULL */, double nu,
                    double dt, int nsteps, double* u, double* v,
                    const int8_t* fixed /* optional [n]: Dirichlet nodes */,
                    const double* dfix /* optional [2][4][n]: their stage derivatives, else 0 */);
/* three dimensions (HERMITE family; k <= 4) */
int or_p3_of_k(int k);
void or_index_table3(int k, int* ea, int* eb, int* ec);
void or_monomials3(int k, double dx, double dy, double dz, double* X);
int or_abfs3(int rbf, double sigma, int k, double dx, double dy, double dz, double* W);
int64_t or_neighbours3_brute(int64_t n, const double* x, const double* y, const double* z,
                             const or_domain3* dom, const double* R, int64_t* row_ptr, int32_t* col);
int or_weights3(int64_t n, const double* x, const double* y, const double* z, const or_domain3* dom,
                const double* R, int k, const int64_t* row_ptr, const int32_t* col, const or_wopts* o,
                double* w /* [nops][nnz], operators in bit order */, int8_t* status, double* resid,
                int8_t* iters);
int or_num_threads(void);
void or_set_num_threads(int t);

#endif
