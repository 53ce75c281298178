/*
 * labfm_oracle.c -- plain, slow, FP64 CPU oracle for the LABFM hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see labfm_oracle.h).  Built with gcc
 * -ffp-contract=off so that every product and sum is rounded as written.
 *
 * The method (King, Lind & Nasar, arXiv:1912.06441):
 *   - neighbours of i: every j != i with |r_j - r_i| < 2h            (Sec. 2)
 *   - offsets d = r_ji / h, monomials X(d), ABFs W(d)              (Sec. 2 eq. 1, Sec. 3.2)
 *   - M = sum_j X(d_j) (x) W(d_j), M Psi^d = C^d, w^d_j = W(d_j).Psi^d   (Sec. 3.1)
 *   - L^d_i(u) = sum_j (u_j - u_i) w^d_ji                           (Sec. 2 eq. general_do)
 * The h-scaling is exact: X(r_ji) has the factor h^|m|, so solving with the
 * scaled offsets and dividing by h^l (l = order of the derivative) gives the
 * same weights as solving in physical units.
 */
#include "labfm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Sec. 3.1: p = (k^2 + 3k)/2 elements for a 2-D scheme of order k.        */
int or_p_of_k(int k) { return (k * k + 3 * k) / 2; }

/* Sec. 3.2: the critical stencil sizes N_crit for k = 2, 4, 6, 8 below which
 * M becomes ill-conditioned.  Odd k take the next even value (reading). */
int or_ncrit(int k) {
    if (k <= 2) return 8;
    if (k <= 4) return 21;
    if (k <= 6) return 37;
    return 57;
}

/* Sec. 2 eq. (1): element m of X is x^a y^b / (a! b!), ordered by total
 * order n = 1..k and, within an order, a = n, n-1, ..., 0. */
void or_index_table(int k, int* ea, int* eb) {
    int m = 0;
    for (int n = 1; n <= k; ++n)
        for (int a = n; a >= 0; --a) {
            ea[m] = a;
            eb[m] = n - a;
            ++m;
        }
}

static double or_factorial(int a) {
    double f = 1.0;
    for (int i = 2; i <= a; ++i) f *= (double)i;
    return f;
}

void or_monomials(int k, double dx, double dy, double* X) {
    int ea[OR_MAXP], eb[OR_MAXP];
    or_index_table(k, ea, eb);
    int p = or_p_of_k(k);
    for (int m = 0; m < p; ++m) {
        double v = 1.0;
        for (int i = 0; i < ea[m]; ++i) v *= dx;
        for (int i = 0; i < eb[m]; ++i) v *= dy;
        X[m] = v / (or_factorial(ea[m]) * or_factorial(eb[m]));
    }
}

/* Physicists' Hermite polynomials: H0 = 1, H1 = 2t, H_{m+1} = 2t H_m - 2m H_{m-1}. */
void or_hermite(int nmax, double t, double* H) {
    H[0] = 1.0;
    if (nmax >= 1) H[1] = 2.0 * t;
    for (int m = 1; m < nmax; ++m) H[m + 1] = 2.0 * t * H[m] - 2.0 * (double)m * H[m - 1];
}

/* ------------------------------------------------------------------------ */
/* Fundamental RBFs of App. A (and Wendland C2), with derivatives in q.     */
/* Each compactly supported RBF is written as c * s^e * P(q), s = 1 - q/2,   */
/* and differentiated with the Leibniz rule.  Constants as printed.          */

static void or_leibniz(double c, int e, const double* P, int degP, double q, double* f) {
    /* (s^e)^(n) = e!/(e-n)! (-1/2)^n s^(e-n) */
    double s = 1.0 - 0.5 * q;
    double se[4], Pd[4];
    for (int nd = 0; nd < 4; ++nd) {
        if (nd > e) {
            se[nd] = 0.0;
        } else {
            double coef = 1.0;
            for (int i = 0; i < nd; ++i) coef *= (double)(e - i) * -0.5;
            double pw = 1.0;
            for (int i = 0; i < e - nd; ++i) pw *= s;
            se[nd] = coef * pw;
        }
        /* nd-th derivative of the polynomial P */
        double acc = 0.0;
        for (int i = nd; i <= degP; ++i) {
            double fall = 1.0;
            for (int t = 0; t < nd; ++t) fall *= (double)(i - t);
            double qp = 1.0;
            for (int t = 0; t < i - nd; ++t) qp *= q;
            acc += P[i] * fall * qp;
        }
        Pd[nd] = acc;
    }
    static const double binom[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
    for (int nd = 0; nd < 4; ++nd) {
        double acc = 0.0;
        for (int i = 0; i <= nd; ++i) acc += binom[nd][i] * se[i] * Pd[nd - i];
        f[nd] = c * acc;
    }
}

int or_rbf_derivs(int rbf, double q, double* f) {
    const double pi = 3.14159265358979323846;
    if (rbf == OR_RBF_GAUSSIAN) {
        /* App. A: W = 9/pi exp(-9 q^2) */
        double g = 9.0 / pi * exp(-9.0 * q * q);
        f[0] = g;
        f[1] = -18.0 * q * g;
        f[2] = (-18.0 + 324.0 * q * q) * g;
        f[3] = (972.0 * q - 5832.0 * q * q * q) * g;
        return 0;
    }
    if (q >= 2.0) {
        f[0] = f[1] = f[2] = f[3] = 0.0;
        return 0;
    }
    if (rbf == OR_RBF_CONE) { /* Sec. 3.2: 3/(4 pi) (1 - q/2) */
        const double P[1] = {1.0};
        or_leibniz(3.0 / (4.0 * pi), 1, P, 0, q, f);
    } else if (rbf == OR_RBF_QUADRATIC) { /* App. A: 3/(16 pi) (q-2)^2 = 3/(16 pi) 4 s^2 */
        const double P[1] = {4.0};
        or_leibniz(3.0 / (16.0 * pi), 2, P, 0, q, f);
    } else if (rbf == OR_RBF_WENDLAND_C6) { /* App. A: 78/(28 pi) s^8 (4q^3 + 6.25q^2 + 4q + 1) */
        const double P[4] = {1.0, 4.0, 6.25, 4.0};
        or_leibniz(78.0 / (28.0 * pi), 8, P, 3, q, f);
    } else if (rbf == OR_RBF_WENDLAND_C2) { /* 2-D Wendland C2, support 2: s^4 (1 + 2q) */
        const double P[2] = {1.0, 2.0};
        or_leibniz(1.0, 4, P, 1, q, f);
    } else {
        return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* PAPER family (Sec. 3.2, App. A).  The dW0/dr part of element (a,b) is     */
/* dW0/dr * d^(a,b) r, and d^(a,b) r = P_ab(x,y) / r^(2n-1) with P_ab a       */
/* homogeneous polynomial of degree n = a+b:                                 */
/*   P_10 = x, P_01 = y,                                                      */
/*   P_(a+1)b = r^2 dP/dx - (2n-1) x P,  P_a(b+1) = r^2 dP/dy - (2n-1) y P.    */
/* Coefficient c[i] multiplies x^(n-i) y^i.                                   */

static double or_Ptab[OR_MAXK + 1][OR_MAXK + 1][OR_MAXK + 1]; /* [a][b][i] */
static void or_pstep(int n, const double* c, int dir, double* out) {
    /* out = r^2 dQ - (2n-1) v Q for Q of degree n, v = x (dir 0) or y (dir 1) */
    double dq[OR_MAXK + 2];
    memset(dq, 0, sizeof(dq));
    /* dQ has degree n-1; dq[i] multiplies x^(n-1-i) y^i */
    for (int i = 0; i <= n; ++i) {
        if (dir == 0) {
            if (n - i >= 1) dq[i] += (double)(n - i) * c[i];
        } else {
            if (i >= 1) dq[i - 1] += (double)i * c[i];
        }
    }
    for (int i = 0; i <= n + 1; ++i) out[i] = 0.0;
    for (int i = 0; i <= n - 1; ++i) {
        out[i] += dq[i];     /* x^2 * x^(n-1-i) y^i -> x^(n+1-i) y^i */
        out[i + 2] += dq[i]; /* y^2 * x^(n-1-i) y^i -> x^(n-1-i) y^(i+2) */
    }
    for (int i = 0; i <= n; ++i) {
        if (dir == 0) out[i] -= (double)(2 * n - 1) * c[i];     /* x * x^(n-i) y^i */
        else out[i + 1] -= (double)(2 * n - 1) * c[i];          /* y * x^(n-i) y^i */
    }
}

__attribute__((constructor)) static void or_build_ptab(void) {
    memset(or_Ptab, 0, sizeof(or_Ptab));
    or_Ptab[1][0][0] = 1.0; /* x */
    or_Ptab[0][1][1] = 1.0; /* y */
    for (int n = 1; n < OR_MAXK; ++n) {
        for (int a = n; a >= 0; --a) {
            int b = n - a;
            /* x-step from (a,b) gives (a+1,b); y-step from (0,n) gives (0,n+1) */
            or_pstep(n, or_Ptab[a][b], 0, or_Ptab[a + 1][b]);
            if (a == 0) or_pstep(n, or_Ptab[0][b], 1, or_Ptab[0][b + 1]);
        }
    }
}

static double or_poly_eval(int n, const double* c, double x, double y) {
    double acc = 0.0;
    for (int i = 0; i <= n; ++i) {
        double t = c[i];
        for (int e = 0; e < n - i; ++e) t *= x;
        for (int e = 0; e < i; ++e) t *= y;
        acc += t;
    }
    return acc;
}

/* App. A, elements 1..9 written out as printed (full derivatives of W0(r)). */
static void or_paper_low(int a, int b, double x, double y, double r, const double* f, double* out) {
    double r2 = r * r, r3 = r2 * r, r4 = r2 * r2, r5 = r4 * r;
    double f1 = f[1], f2 = f[2], f3 = f[3];
    int n = a + b;
    double v = 0.0;
    if (n == 1) {
        v = (a == 1) ? f1 * x / r : f1 * y / r;
    } else if (n == 2) {
        if (a == 2) v = f1 * y * y / r3 + f2 * x * x / r2;
        else if (a == 1) v = -f1 * x * y / r3 + f2 * x * y / r2;
        else v = f1 * x * x / r3 + f2 * y * y / r2;
    } else { /* n == 3 */
        if (a == 3)
            v = f1 * (-3.0 * x * y * y) / r5 + f2 * (3.0 * x * y * y) / r4 + f3 * x * x * x / r3;
        else if (a == 2)
            v = f1 * (2.0 * x * x * y - y * y * y) / r5 + f2 * (y * y * y - 2.0 * x * x * y) / r4 +
                f3 * x * x * y / r3;
        else if (a == 1)
            v = f1 * (2.0 * x * y * y - x * x * x) / r5 + f2 * (x * x * x - 2.0 * x * y * y) / r4 +
                f3 * x * y * y / r3;
        else
            v = f1 * (-3.0 * x * x * y) / r5 + f2 * (3.0 * x * x * y) / r4 + f3 * y * y * y / r3;
    }
    *out = v;
}

/* ABF vector W(d) for offset d = (dx, dy) in units of h.  Returns nonzero if
 * the ABFs are undefined at this offset (PAPER families at d = 0).
 * PAPER: full derivatives of W0 up to total order 3, then only the dW0/dr
 * term (App. A).  PAPER_D1: only the dW0/dr term in every element (the App. A
 * truncation applied from the first element on). */
int or_abfs(int family, int rbf, double sigma, int k, double dx, double dy, double* W) {
    int ea[OR_MAXP], eb[OR_MAXP];
    or_index_table(k, ea, eb);
    int p = or_p_of_k(k);
    double q = sqrt(dx * dx + dy * dy);
    double f[4];
    if (or_rbf_derivs(rbf, q, f) != 0) return -1;
    if (family == OR_ABF_HERMITE) {
        double Hx[OR_MAXK + 1], Hy[OR_MAXK + 1];
        or_hermite(k, sigma * dx, Hx);
        or_hermite(k, sigma * dy, Hy);
        for (int m = 0; m < p; ++m) W[m] = Hx[ea[m]] * Hy[eb[m]] * f[0];
        return 0;
    }
    if (q == 0.0) return 1;
    for (int m = 0; m < p; ++m) {
        int a = ea[m], b = eb[m], n = a + b;
        if (family == OR_ABF_PAPER && n <= 3) {
            or_paper_low(a, b, dx, dy, q, f, &W[m]);
        } else {
            double den = 1.0;
            for (int e = 0; e < 2 * n - 1; ++e) den *= q;
            W[m] = f[1] * or_poly_eval(n, or_Ptab[a][b], dx, dy) / den;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets (Sec. 2): j != i with squared distance < R_i^2, periodic   */
/* axes by minimum image, ascending j.  Radius growth (reading of Sec. 3.2's */
/* critical stencil size): R_i <- 1.1 R_i until N_i >= N_crit(k_i).          */

static inline double or_wrap(double d, double L, int per) {
    if (!per) return d;
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

static int or_cmp_i32(const void* a, const void* b) {
    int32_t u = *(const int32_t*)a, v = *(const int32_t*)b;
    return (u > v) - (u < v);
}

static int64_t or_count_brute(int64_t i, int64_t n, const double* x, const double* y,
                              const or_domain* dom, double R, int32_t* out) {
    double Lx = dom->hi[0] - dom->lo[0], Ly = dom->hi[1] - dom->lo[1];
    double R2 = R * R;
    int64_t c = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = or_wrap(x[j] - x[i], Lx, dom->periodic[0]);
        double dy = or_wrap(y[j] - y[i], Ly, dom->periodic[1]);
        double d2 = dx * dx + dy * dy;
        if (d2 < R2) {
            if (out) out[c] = (int32_t)j;
            ++c;
        }
    }
    return c;
}

int64_t or_neighbours_brute(int64_t n, const double* x, const double* y, const or_domain* dom,
                            double* R, const int8_t* order, int grow, int max_grow,
                            int64_t* row_ptr, int32_t* col) {
    if (!col) {
        row_ptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t c = or_count_brute(i, n, x, y, dom, R[i], NULL);
            if (grow) {
                int it = 0;
                while (c < or_ncrit(order[i]) && it < max_grow) {
                    R[i] = R[i] * 1.1;
                    c = or_count_brute(i, n, x, y, dom, R[i], NULL);
                    ++it;
                }
            }
            row_ptr[i + 1] = row_ptr[i] + c;
        }
        return row_ptr[n];
    }
    for (int64_t i = 0; i < n; ++i) or_count_brute(i, n, x, y, dom, R[i], col + row_ptr[i]);
    return row_ptr[n];
}

/* Same sets through a uniform bucket grid (an acceleration only). */
typedef struct {
    int ncx, ncy;
    double wx, wy;
    int64_t* start; /* ncx*ncy+1 */
    int32_t* idx;
} or_grid;

static int or_cell_of(double v, double lo, double w, int nc) {
    int c = (int)floor((v - lo) / w);
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
    return c;
}

static void or_grid_build(or_grid* g, int64_t n, const double* x, const double* y,
                          const or_domain* dom, double cell) {
    double Lx = dom->hi[0] - dom->lo[0], Ly = dom->hi[1] - dom->lo[1];
    g->ncx = (int)floor(Lx / cell);
    g->ncy = (int)floor(Ly / cell);
    if (g->ncx < 1) g->ncx = 1;
    if (g->ncy < 1) g->ncy = 1;
    g->wx = Lx / g->ncx;
    g->wy = Ly / g->ncy;
    int64_t nc = (int64_t)g->ncx * g->ncy;
    g->start = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
    g->idx = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int* cid = (int*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    for (int64_t i = 0; i < n; ++i) {
        int cx = or_cell_of(x[i], dom->lo[0], g->wx, g->ncx);
        int cy = or_cell_of(y[i], dom->lo[1], g->wy, g->ncy);
        cid[i] = cy * g->ncx + cx;
        g->start[cid[i] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) g->start[c + 1] += g->start[c];
    int64_t* fillp = (int64_t*)malloc((size_t)nc * sizeof(int64_t) + 1);
    memcpy(fillp, g->start, (size_t)nc * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) g->idx[fillp[cid[i]]++] = (int32_t)i;
    free(fillp);
    free(cid);
}

static void or_grid_free(or_grid* g) {
    free(g->start);
    free(g->idx);
}

static int64_t or_count_cells(int64_t i, const double* x, const double* y, const or_domain* dom,
                              const or_grid* g, double R, int32_t* out) {
    double Lx = dom->hi[0] - dom->lo[0], Ly = dom->hi[1] - dom->lo[1];
    double R2 = R * R;
    int cx = or_cell_of(x[i], dom->lo[0], g->wx, g->ncx);
    int cy = or_cell_of(y[i], dom->lo[1], g->wy, g->ncy);
    int rx = (int)ceil(R / g->wx), ry = (int)ceil(R / g->wy);
    int x0, x1, y0, y1;
    if (dom->periodic[0] && 2 * rx + 1 >= g->ncx) { x0 = 0; x1 = g->ncx - 1; }
    else if (dom->periodic[0]) { x0 = cx - rx; x1 = cx + rx; }
    else { x0 = cx - rx < 0 ? 0 : cx - rx; x1 = cx + rx >= g->ncx ? g->ncx - 1 : cx + rx; }
    if (dom->periodic[1] && 2 * ry + 1 >= g->ncy) { y0 = 0; y1 = g->ncy - 1; }
    else if (dom->periodic[1]) { y0 = cy - ry; y1 = cy + ry; }
    else { y0 = cy - ry < 0 ? 0 : cy - ry; y1 = cy + ry >= g->ncy ? g->ncy - 1 : cy + ry; }
    int64_t c = 0;
    for (int yy = y0; yy <= y1; ++yy) {
        int ccy = ((yy % g->ncy) + g->ncy) % g->ncy;
        for (int xx = x0; xx <= x1; ++xx) {
            int ccx = ((xx % g->ncx) + g->ncx) % g->ncx;
            int64_t cell = (int64_t)ccy * g->ncx + ccx;
            for (int64_t s = g->start[cell]; s < g->start[cell + 1]; ++s) {
                int32_t j = g->idx[s];
                if (j == i) continue;
                double dx = or_wrap(x[j] - x[i], Lx, dom->periodic[0]);
                double dy = or_wrap(y[j] - y[i], Ly, dom->periodic[1]);
                double d2 = dx * dx + dy * dy;
                if (d2 < R2) {
                    if (out) out[c] = j;
                    ++c;
                }
            }
        }
    }
    if (out) qsort(out, (size_t)c, sizeof(int32_t), or_cmp_i32);
    return c;
}

int64_t or_neighbours_cells(int64_t n, const double* x, const double* y, const or_domain* dom,
                            double* R, const int8_t* order, int grow, int max_grow,
                            int64_t* row_ptr, int32_t* col) {
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i) rmax = R[i] > rmax ? R[i] : rmax;
    if (rmax <= 0.0) rmax = 1.0;
    or_grid g;
    or_grid_build(&g, n, x, y, dom, rmax);
    if (!col) {
        int64_t* cnt = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            int64_t c = or_count_cells(i, x, y, dom, &g, R[i], NULL);
            if (grow) {
                int it = 0;
                while (c < or_ncrit(order[i]) && it < max_grow) {
                    R[i] = R[i] * 1.1;
                    c = or_count_cells(i, x, y, dom, &g, R[i], NULL);
                    ++it;
                }
            }
            cnt[i] = c;
        }
        row_ptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
        free(cnt);
    } else {
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) or_count_cells(i, x, y, dom, &g, R[i], col + row_ptr[i]);
    }
    or_grid_free(&g);
    return row_ptr[n];
}

/* ------------------------------------------------------------------------ */
/* Target vectors C^d (Sec. 2 and Sec. 4.2), in element order of X.          */
/* x: e1; y: e2; Laplacian: e3 + e5; -nabla^4: -(e10 + 2 e12 + e14);        */
/* nabla^6: e21 + 3 e23 + 3 e25 + e27 (1-based).  l = derivative order.      */
static int or_target(unsigned op, int p, double* C, int* l) {
    for (int m = 0; m < p; ++m) C[m] = 0.0;
    switch (op) {
        case OR_OP_DX: C[0] = 1.0; *l = 1; return 0;
        case OR_OP_DY: C[1] = 1.0; *l = 1; return 0;
        case OR_OP_LAP: C[2] = 1.0; C[4] = 1.0; *l = 2; return 0;
        case OR_OP_BIHARM:
            if (p < 14) return -1;
            C[9] = -1.0; C[11] = -2.0; C[13] = -1.0; *l = 4; return 0;
        case OR_OP_TRIHARM:
            if (p < 27) return -1;
            C[20] = 1.0; C[22] = 3.0; C[24] = 3.0; C[26] = 1.0; *l = 6; return 0;
    }
    return -1;
}

/* Target vectors C^d of the requested operators, [nops][p] for order k. */
int or_targets(unsigned ops, int k, double* C) {
    int p = or_p_of_k(k), op_i = 0, l;
    for (int b = 0; b < 5; ++b) {
        if (!((ops >> b) & 1u)) continue;
        if (or_target(1u << b, p, C + (size_t)op_i * p, &l) != 0) return -1;
        ++op_i;
    }
    return 0;
}

/* Dense LU with partial pivoting on a p x p row-major matrix, after row then
 * column max-abs equilibration (a reading: the paper does not name a solver).
 * Ties in the pivot search go to the lowest row index. */
typedef struct {
    int p;
    double A[OR_MAXP * OR_MAXP];
    int piv[OR_MAXP];
    double rs[OR_MAXP], cs[OR_MAXP];
} or_lu;

static int or_lu_factor(or_lu* F, const double* M, int p) {
    F->p = p;
    memcpy(F->A, M, sizeof(double) * (size_t)p * p);
    for (int r = 0; r < p; ++r) {
        double mx = 0.0;
        for (int c = 0; c < p; ++c) mx = fmax(mx, fabs(F->A[r * p + c]));
        if (!(mx > 0.0) || !isfinite(mx)) return -1;
        F->rs[r] = 1.0 / mx;
        for (int c = 0; c < p; ++c) F->A[r * p + c] *= F->rs[r];
    }
    for (int c = 0; c < p; ++c) {
        double mx = 0.0;
        for (int r = 0; r < p; ++r) mx = fmax(mx, fabs(F->A[r * p + c]));
        if (!(mx > 0.0)) return -1;
        F->cs[c] = 1.0 / mx;
        for (int r = 0; r < p; ++r) F->A[r * p + c] *= F->cs[c];
    }
    for (int kk = 0; kk < p; ++kk) {
        int pr = kk;
        double best = fabs(F->A[kk * p + kk]);
        for (int r = kk + 1; r < p; ++r) {
            double v = fabs(F->A[r * p + kk]);
            if (v > best) { best = v; pr = r; }
        }
        if (!(best > 0.0) || !isfinite(best)) return -1;
        F->piv[kk] = pr;
        if (pr != kk)
            for (int c = 0; c < p; ++c) {
                double t = F->A[kk * p + c];
                F->A[kk * p + c] = F->A[pr * p + c];
                F->A[pr * p + c] = t;
            }
        double d = F->A[kk * p + kk];
        for (int r = kk + 1; r < p; ++r) {
            double l = F->A[r * p + kk] / d;
            F->A[r * p + kk] = l;
            for (int c = kk + 1; c < p; ++c) F->A[r * p + c] -= l * F->A[kk * p + c];
        }
    }
    return 0;
}

/* Solve M z = b with the factors: z = D_c U^-1 L^-1 P D_r b. */
static void or_lu_solve(const or_lu* F, const double* b, double* z) {
    int p = F->p;
    double t[OR_MAXP];
    for (int r = 0; r < p; ++r) t[r] = b[r] * F->rs[r];
    for (int kk = 0; kk < p; ++kk) {
        int pr = F->piv[kk];
        if (pr != kk) { double s = t[kk]; t[kk] = t[pr]; t[pr] = s; }
    }
    for (int r = 0; r < p; ++r) {
        double acc = t[r];
        for (int c = 0; c < r; ++c) acc -= F->A[r * p + c] * t[c];
        t[r] = acc;
    }
    for (int r = p - 1; r >= 0; --r) {
        double acc = t[r];
        for (int c = r + 1; c < p; ++c) acc -= F->A[r * p + c] * t[c];
        t[r] = acc / F->A[r * p + r];
    }
    for (int r = 0; r < p; ++r) z[r] = t[r] * F->cs[r];
}

/* 1-norm condition number of the equilibrated matrix (explicit inverse). */
static double or_cond1(const or_lu* F) {
    int p = F->p;
    /* rebuild the equilibrated matrix from L U with row pivots undone */
    double LU[OR_MAXP * OR_MAXP];
    for (int r = 0; r < p; ++r)
        for (int c = 0; c < p; ++c) {
            double acc = 0.0;
            int kmax = r < c ? r : c;
            for (int kk = 0; kk <= kmax; ++kk) {
                double l = (kk == r) ? 1.0 : F->A[r * p + kk];
                acc += l * F->A[kk * p + c];
            }
            LU[r * p + c] = acc;
        }
    for (int kk = p - 1; kk >= 0; --kk) {
        int pr = F->piv[kk];
        if (pr != kk)
            for (int c = 0; c < p; ++c) {
                double t = LU[kk * p + c];
                LU[kk * p + c] = LU[pr * p + c];
                LU[pr * p + c] = t;
            }
    }
    double nA = 0.0;
    for (int c = 0; c < p; ++c) {
        double s = 0.0;
        for (int r = 0; r < p; ++r) s += fabs(LU[r * p + c]);
        nA = fmax(nA, s);
    }
    /* inverse of the equilibrated matrix: columns e_c through the factors */
    double nI = 0.0;
    for (int c = 0; c < p; ++c) {
        double t[OR_MAXP];
        for (int r = 0; r < p; ++r) t[r] = (r == c) ? 1.0 : 0.0;
        for (int kk = 0; kk < p; ++kk) {
            int pr = F->piv[kk];
            if (pr != kk) { double s = t[kk]; t[kk] = t[pr]; t[pr] = s; }
        }
        for (int r = 0; r < p; ++r) {
            double acc = t[r];
            for (int q = 0; q < r; ++q) acc -= F->A[r * p + q] * t[q];
            t[r] = acc;
        }
        for (int r = p - 1; r >= 0; --r) {
            double acc = t[r];
            for (int q = r + 1; q < p; ++q) acc -= F->A[r * p + q] * t[q];
            t[r] = acc / F->A[r * p + r];
        }
        double s = 0.0;
        for (int r = 0; r < p; ++r) s += fabs(t[r]);
        nI = fmax(nI, s);
    }
    return nA * nI;
}

static int or_nops(unsigned ops) {
    int c = 0;
    for (int b = 0; b < 5; ++b) c += (ops >> b) & 1u;
    return c;
}

/* One node: scaled offsets (dx/h, dy/h) of its N neighbours in ascending j.
 * Writes the scaled weights what[o][j] (unscaling by h^l is the caller's),
 * the final moment residual max_o ||C^o - X^T w^o||_inf and the number of
 * refinement updates.  Refinement (a reading, for FP64 round-off at k = 8):
 *   r = C - X^T w;  stop if ||r|| <= tol_stop;  w += W (M^-1 r). */
/* One node system.  psi (optional, [nops][p]) receives the ABF coefficients
 * Psi^d of eq. (lsys) including every refinement correction, so that
 * w = W Psi holds for the returned weights. */
static int node_weights_impl(int k, int N, const double* dxh, const double* dyh, const or_wopts* o,
                             double* what, double* resid, int* iters, double* Mhat, double* cond1,
                             double* psi) {
    int p = or_p_of_k(k);
    int nops = or_nops(o->ops);
    *resid = INFINITY;
    *iters = 0;
    if (cond1) *cond1 = INFINITY;
    for (int i = 0; i < nops * N; ++i) what[i] = 0.0;
    if (psi)
        for (int i = 0; i < nops * p; ++i) psi[i] = 0.0;
    if (k < 1 || k > OR_MAXK) return OR_ST_ORDER_TOO_LOW;
    {
        int op_i = 0;
        for (int b = 0; b < 5; ++b) {
            if (!((o->ops >> b) & 1u)) continue;
            double Ct[OR_MAXP];
            int l;
            if (or_target(1u << b, p, Ct, &l) != 0) return OR_ST_ORDER_TOO_LOW;
            ++op_i;
        }
    }
    if (N < p) return OR_ST_TOO_FEW;
    if (N > OR_NMAX) return OR_ST_TOO_MANY;
    double* X = (double*)malloc(sizeof(double) * (size_t)N * p);
    double* W = (double*)malloc(sizeof(double) * (size_t)N * p);
    for (int j = 0; j < N; ++j) {
        or_monomials(k, dxh[j], dyh[j], X + (size_t)j * p);
        if (or_abfs(o->family, o->rbf, o->sigma, k, dxh[j], dyh[j], W + (size_t)j * p) != 0) {
            free(X);
            free(W);
            return OR_ST_DEGENERATE;
        }
    }
    /* eq. (disc_form): M[m][n] = sum_j X_m(d_j) W_n(d_j) */
    double M[OR_MAXP * OR_MAXP];
    for (int m = 0; m < p; ++m)
        for (int nn = 0; nn < p; ++nn) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j) acc += X[(size_t)j * p + m] * W[(size_t)j * p + nn];
            M[m * p + nn] = acc;
        }
    if (Mhat) memcpy(Mhat, M, sizeof(double) * (size_t)p * p);
    or_lu F;
    if (or_lu_factor(&F, M, p) != 0) {
        free(X);
        free(W);
        return OR_ST_SINGULAR;
    }
    if (cond1) *cond1 = or_cond1(&F);
    double worst = 0.0;
    int maxit = 0;
    int op_i = 0;
    for (int b = 0; b < 5; ++b) {
        if (!((o->ops >> b) & 1u)) continue;
        double C[OR_MAXP], Psi[OR_MAXP], r[OR_MAXP];
        int l;
        or_target(1u << b, p, C, &l);
        double* w = what + (size_t)op_i * N;
        /* eq. (lsys) then eq. (w_abf) */
        or_lu_solve(&F, C, Psi);
        for (int j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int nn = 0; nn < p; ++nn) acc += W[(size_t)j * p + nn] * Psi[nn];
            w[j] = acc;
        }
        int it = 0;
        double res = 0.0;
        for (;;) {
            res = 0.0;
            for (int m = 0; m < p; ++m) {
                double acc = 0.0;
                for (int j = 0; j < N; ++j) acc += X[(size_t)j * p + m] * w[j];
                r[m] = C[m] - acc;
                res = fmax(res, fabs(r[m]));
            }
            if (!(res > o->tol_stop) || it >= o->max_iters) break;
            double dPsi[OR_MAXP];
            or_lu_solve(&F, r, dPsi);
            for (int nn = 0; nn < p; ++nn) Psi[nn] += dPsi[nn];
            for (int j = 0; j < N; ++j) {
                double acc = 0.0;
                for (int nn = 0; nn < p; ++nn) acc += W[(size_t)j * p + nn] * dPsi[nn];
                w[j] += acc;
            }
            ++it;
        }
        if (!isfinite(res)) res = INFINITY;
        if (psi) memcpy(psi + (size_t)op_i * p, Psi, sizeof(double) * (size_t)p);
        worst = fmax(worst, res);
        if (it > maxit) maxit = it;
        ++op_i;
    }
    free(X);
    free(W);
    *resid = worst;
    *iters = maxit;
    if (!(worst <= 1e-10)) return OR_ST_NOT_CONVERGED;
    return OR_ST_OK;
}

int or_node_weights(int k, int N, const double* dxh, const double* dyh, const or_wopts* o,
                    double* what, double* resid, int* iters, double* Mhat, double* cond1) {
    return node_weights_impl(k, N, dxh, dyh, o, what, resid, iters, Mhat, cond1, NULL);
}

/* ABF coefficients of a batch of stencils given by scaled offsets:
 * stencil s has N[s] <= Nmax offsets dxh[s*Nmax + j], dyh[s*Nmax + j]; psi
 * [n][nops][p] (p of order k), status[n], resid[n], Mhat (optional) [n][p][p]
 * the moment matrices of eq. (disc_form). */
void or_stencils_psi(int64_t n, int k, int Nmax, const int32_t* N, const double* dxh, const double* dyh,
                     const or_wopts* o, double* psi, int8_t* status, double* resid, double* Mhat) {
    int nops = or_nops(o->ops);
    int p = or_p_of_k(k);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < n; ++s) {
        double* wh = (double*)malloc(sizeof(double) * (size_t)(N[s] > 0 ? N[s] : 1) * nops);
        double res;
        int it;
        status[s] = (int8_t)node_weights_impl(k, N[s], dxh + (size_t)s * Nmax, dyh + (size_t)s * Nmax, o, wh, &res,
                                              &it, Mhat ? Mhat + (size_t)s * p * p : NULL, NULL,
                                              psi + (size_t)s * nops * p);
        resid[s] = res;
        free(wh);
    }
}

int or_weights(int64_t n, const double* x, const double* y, const or_domain* dom, const double* R,
               const int8_t* order, const int64_t* row_ptr, const int32_t* col, const or_wopts* o,
               double* w, int8_t* status, double* resid, int8_t* iters) {
    int nops = or_nops(o->ops);
    int64_t nnz = row_ptr[n];
    double Lx = dom->hi[0] - dom->lo[0], Ly = dom->hi[1] - dom->lo[1];
    int nbad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nbad)
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = row_ptr[i];
        int N = (int)(row_ptr[i + 1] - s);
        double h = 0.5 * R[i];
        double* dxh = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        double* dyh = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        double* wh = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * nops);
        for (int j = 0; j < N; ++j) {
            int32_t c = col[s + j];
            dxh[j] = or_wrap(x[c] - x[i], Lx, dom->periodic[0]) / h;
            dyh[j] = or_wrap(y[c] - y[i], Ly, dom->periodic[1]) / h;
        }
        double res;
        int it;
        int st = or_node_weights(order[i], N, dxh, dyh, o, wh, &res, &it, NULL, NULL);
        int op_i = 0;
        for (int b = 0; b < 5; ++b) {
            if (!((o->ops >> b) & 1u)) continue;
            double C[OR_MAXP];
            int l = 1;
            or_target(1u << b, OR_MAXP, C, &l);
            double hl = 1.0;
            for (int e = 0; e < l; ++e) hl *= h;
            for (int j = 0; j < N; ++j)
                w[(size_t)op_i * nnz + s + j] =
                    (st == OR_ST_OK || st == OR_ST_NOT_CONVERGED) ? wh[(size_t)op_i * N + j] / hl : 0.0;
            ++op_i;
        }
        status[i] = (int8_t)st;
        resid[i] = res;
        iters[i] = (int8_t)it;
        if (st != OR_ST_OK) nbad++;
        free(dxh);
        free(dyh);
        free(wh);
    }
    return nbad;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2 eq. (general_do): L_i(u) = sum_j (u_j - u_i) w_ji, ascending j.    */
void or_apply(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* w,
              const double* u, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t s = row_ptr[i]; s < row_ptr[i + 1]; ++s) acc += (u[col[s]] - u[i]) * w[s];
        out[i] = acc;
    }
}

/* Linear combination of weight sets (exact by linearity of C^d). */
void or_combine(int64_t nnz, int nsets, const double* w, const double* coef, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nnz; ++s) {
        double acc = 0.0;
        for (int k = 0; k < nsets; ++k) acc += coef[k] * w[(size_t)k * nnz + s];
        out[s] = acc;
    }
}

/* Classical RK4 (Sec. 5.1) on du/dt = L_lin(u) - gamma B(B(u)), where B is
 * the biharmonic stencil (B o B approximates nabla^8) or absent. */
static void or_rhs(int64_t n, const int64_t* rp, const int32_t* col, const double* w_lin,
                   const double* w_bh, double gamma, const double* u, double* f, double* t1,
                   double* t2) {
    or_apply(n, rp, col, w_lin, u, f);
    if (w_bh) {
        or_apply(n, rp, col, w_bh, u, t1);
        or_apply(n, rp, col, w_bh, t1, t2);
        for (int64_t i = 0; i < n; ++i) f[i] = f[i] - gamma * t2[i];
    }
}

/* Dirichlet nodes (fixed[i] != 0, Sec. 5.1): u is prescribed there, so its
 * time derivative is zero and only the other nodes are advanced. */
static void or_pin(int64_t n, const int8_t* fixed, double* k) {
    if (!fixed) return;
    for (int64_t i = 0; i < n; ++i)
        if (fixed[i]) k[i] = 0.0;
}

void or_rk4(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* w_lin,
            const double* w_bh, double gamma, double dt, int nsteps, double* u, const int8_t* fixed) {
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *k1 = malloc(sz), *k2 = malloc(sz), *k3 = malloc(sz), *k4 = malloc(sz);
    double *us = malloc(sz), *t1 = malloc(sz), *t2 = malloc(sz);
    for (int st = 0; st < nsteps; ++st) {
        or_rhs(n, row_ptr, col, w_lin, w_bh, gamma, u, k1, t1, t2);
        or_pin(n, fixed, k1);
        for (int64_t i = 0; i < n; ++i) us[i] = u[i] + 0.5 * dt * k1[i];
        or_rhs(n, row_ptr, col, w_lin, w_bh, gamma, us, k2, t1, t2);
        or_pin(n, fixed, k2);
        for (int64_t i = 0; i < n; ++i) us[i] = u[i] + 0.5 * dt * k2[i];
        or_rhs(n, row_ptr, col, w_lin, w_bh, gamma, us, k3, t1, t2);
        or_pin(n, fixed, k3);
        for (int64_t i = 0; i < n; ++i) us[i] = u[i] + dt * k3[i];
        or_rhs(n, row_ptr, col, w_lin, w_bh, gamma, us, k4, t1, t2);
        or_pin(n, fixed, k4);
        for (int64_t i = 0; i < n; ++i)
            u[i] = u[i] + dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    free(k1); free(k2); free(k3); free(k4); free(us); free(t1); free(t2);
}

/* Viscous Burgers' equation (Sec. 5.3, eq. burgers) for the velocity (u, v):
 *   du/dt = -(u L^x(u) + v L^y(u)) + nu L^L(u) + L^hv(u),
 *   dv/dt = -(u L^x(v) + v L^y(v)) + nu L^L(v) + L^hv(v),
 * nu = 1/Re, L^hv an optional hyperviscosity operator whose coefficient is
 * part of its weights (Sec. 4.2), each L by eq. (general_do).  Classical RK4
 * (Sec. 5.1); nodes with fixed[i] != 0 take, at RK4 stage q, the derivatives
 * dfix[q * n + i] (for u) and dfix[(4 + q) * n + i] (for v) in place of the
 * right-hand side: the time derivative of a prescribed boundary solution
 * (Sec. 5.3, travelling wave), or zero when dfix is NULL (values held). */
static void or_burgers_rhs(int64_t n, const int64_t* rp, const int32_t* col, const double* wx,
                           const double* wy, const double* wl, const double* whv, double nu,
                           const double* u, const double* v, double* ku, double* kv, double* t) {
    /* t: 8 scratch arrays of n: L^x u, L^y u, L^L u, L^hv u, then the same of v */
    const double* f[2] = {u, v};
    for (int c = 0; c < 2; ++c) {
        double* o = t + (size_t)4 * c * n;
        or_apply(n, rp, col, wx, f[c], o);
        or_apply(n, rp, col, wy, f[c], o + n);
        or_apply(n, rp, col, wl, f[c], o + 2 * n);
        if (whv) or_apply(n, rp, col, whv, f[c], o + 3 * n);
        else for (int64_t i = 0; i < n; ++i) o[3 * n + i] = 0.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        const double* a = t;
        const double* b = t + (size_t)4 * n;
        ku[i] = -(u[i] * a[i] + v[i] * a[n + i]) + nu * a[2 * n + i] + a[3 * n + i];
        kv[i] = -(u[i] * b[i] + v[i] * b[n + i]) + nu * b[2 * n + i] + b[3 * n + i];
    }
}

void or_burgers_rk4(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* wx,
                    const double* wy, const double* wl, const double* whv, double nu, double dt,
                    int nsteps, double* u, double* v, const int8_t* fixed, const double* dfix) {
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *ku[4], *kv[4];
    for (int q = 0; q < 4; ++q) { ku[q] = malloc(sz); kv[q] = malloc(sz); }
    double *us = malloc(sz), *vs = malloc(sz), *t = malloc(8 * sz);
    const double c[4] = {0.0, 0.5, 0.5, 1.0}; /* stage q is evaluated at u + c[q] dt k_(q-1) */
    for (int st = 0; st < nsteps; ++st) {
        for (int q = 0; q < 4; ++q) {
            const double *uq = u, *vq = v;
            if (q > 0) {
                for (int64_t i = 0; i < n; ++i) {
                    us[i] = u[i] + c[q] * dt * ku[q - 1][i];
                    vs[i] = v[i] + c[q] * dt * kv[q - 1][i];
                }
                uq = us;
                vq = vs;
            }
            or_burgers_rhs(n, row_ptr, col, wx, wy, wl, whv, nu, uq, vq, ku[q], kv[q], t);
            if (fixed && dfix) {
                for (int64_t i = 0; i < n; ++i)
                    if (fixed[i]) {
                        ku[q][i] = dfix[(size_t)q * n + i];
                        kv[q][i] = dfix[(size_t)(4 + q) * n + i];
                    }
            } else {
                or_pin(n, fixed, ku[q]);
                or_pin(n, fixed, kv[q]);
            }
        }
        for (int64_t i = 0; i < n; ++i) {
            u[i] = u[i] + dt / 6.0 * (ku[0][i] + 2.0 * ku[1][i] + 2.0 * ku[2][i] + ku[3][i]);
            v[i] = v[i] + dt / 6.0 * (kv[0][i] + 2.0 * kv[1][i] + 2.0 * kv[2][i] + kv[3][i]);
        }
    }
    for (int q = 0; q < 4; ++q) { free(ku[q]); free(kv[q]); }
    free(us); free(vs); free(t);
}

/* ======================================================================== */
/* Three dimensions.  Sec. 3.1: in 3-D, p is the sum of the triangular       */
/* numbers 2..k+1 (3, 9, 19, 34, 55, 83 for k = 1..6).  Element order (a     */
/* reading):                                                                 */
/* total order n = 1..k; within n, a = n..0, then b = n-a..0, c = n-a-b.      */
/* X_m = x^a y^b z^c / (a! b! c!) (the Taylor coefficients, as eq. (1));      */
/* ABFs of the HERMITE family H_a(s x) H_b(s y) H_c(s z) phi(|d|).            */

int or_p3_of_k(int k) {
    int p = 0;
    for (int m = 2; m <= k + 1; ++m) p += m * (m + 1) / 2;
    return p;
}

void or_index_table3(int k, int* ea, int* eb, int* ec) {
    if (k < 1 || k > OR_MAXK3) return;
    int m = 0;
    for (int n = 1; n <= k; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                ea[m] = a;
                eb[m] = b;
                ec[m] = n - a - b;
                ++m;
            }
}

void or_monomials3(int k, double dx, double dy, double dz, double* X) {
    if (k < 1 || k > OR_MAXK3) return;
    int ea[OR_MAXP], eb[OR_MAXP], ec[OR_MAXP];
    or_index_table3(k, ea, eb, ec);
    int p = or_p3_of_k(k);
    for (int m = 0; m < p; ++m) {
        double v = 1.0;
        for (int e = 0; e < ea[m]; ++e) v *= dx;
        for (int e = 0; e < eb[m]; ++e) v *= dy;
        for (int e = 0; e < ec[m]; ++e) v *= dz;
        X[m] = v / (or_factorial(ea[m]) * or_factorial(eb[m]) * or_factorial(ec[m]));
    }
}

int or_abfs3(int rbf, double sigma, int k, double dx, double dy, double dz, double* W) {
    if (k < 1 || k > OR_MAXK3) return -1;
    int ea[OR_MAXP], eb[OR_MAXP], ec[OR_MAXP];
    or_index_table3(k, ea, eb, ec);
    int p = or_p3_of_k(k);
    double q = sqrt(dx * dx + dy * dy + dz * dz);
    double f[4];
    if (or_rbf_derivs(rbf, q, f) != 0) return -1;
    double Hx[OR_MAXK + 1], Hy[OR_MAXK + 1], Hz[OR_MAXK + 1];
    or_hermite(k, sigma * dx, Hx);
    or_hermite(k, sigma * dy, Hy);
    or_hermite(k, sigma * dz, Hz);
    for (int m = 0; m < p; ++m) W[m] = Hx[ea[m]] * Hy[eb[m]] * Hz[ec[m]] * f[0];
    return 0;
}

/* 3-D targets: d/dx e(1,0,0), d/dy e(0,1,0), d/dz e(0,0,1) (elements 1, 2, 3),
 * Laplacian e(2,0,0) + e(0,2,0) + e(0,0,2) (elements 4, 7, 9; 1-based). */
static int or_target3(unsigned op, int p, double* C, int* l) {
    for (int m = 0; m < p; ++m) C[m] = 0.0;
    switch (op) {
        case OR_OP_DX: C[0] = 1.0; *l = 1; return 0;
        case OR_OP_DY: C[1] = 1.0; *l = 1; return 0;
        case OR_OP_DZ: C[2] = 1.0; *l = 1; return 0;
        case OR_OP_LAP:
            if (p < 9) return -1;
            C[3] = 1.0; C[6] = 1.0; C[8] = 1.0; *l = 2; return 0;
    }
    return -1;
}

/* operators of a 3-D request, in increasing bit order (DX, DY, LAP, DZ) */
static int or_ops3(unsigned ops, unsigned* list) {
    int c = 0;
    for (int b = 0; b < 6; ++b)
        if ((ops >> b) & 1u) list[c++] = 1u << b;
    return c;
}

/* Neighbours in 3-D by brute force: j != i, squared distance (summed x, y, z
 * in that order) < R_i^2, minimum image on periodic axes, ascending j.  col
 * NULL: row_ptr only. */
int64_t or_neighbours3_brute(int64_t n, const double* x, const double* y, const double* z,
                             const or_domain3* dom, const double* R, int64_t* row_ptr, int32_t* col) {
    double L[3] = {dom->hi[0] - dom->lo[0], dom->hi[1] - dom->lo[1], dom->hi[2] - dom->lo[2]};
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double R2 = R[i] * R[i];
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = or_wrap(x[j] - x[i], L[0], dom->periodic[0]);
            double dy = or_wrap(y[j] - y[i], L[1], dom->periodic[1]);
            double dz = or_wrap(z[j] - z[i], L[2], dom->periodic[2]);
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < R2) {
                if (col) col[row_ptr[i] + c] = (int32_t)j;
                ++c;
            }
        }
        cnt[i] = c;
    }
    if (!col) {
        row_ptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    }
    free(cnt);
    return row_ptr[n];
}

/* One 3-D node system: the steps of node_weights_impl with the 3-D basis. */
static int node_weights3(int k, int N, const double* dxh, const double* dyh, const double* dzh,
                         const or_wopts* o, double* what, double* resid, int* iters) {
    int p = or_p3_of_k(k);
    unsigned list[6];
    int nops = or_ops3(o->ops, list);
    *resid = INFINITY;
    *iters = 0;
    for (int i = 0; i < nops * N; ++i) what[i] = 0.0;
    if (k < 1 || k > OR_MAXK3) return OR_ST_ORDER_TOO_LOW;
    for (int d = 0; d < nops; ++d) {
        double Ct[OR_MAXP];
        int l;
        if (or_target3(list[d], p, Ct, &l) != 0) return OR_ST_ORDER_TOO_LOW;
    }
    if (N < p) return OR_ST_TOO_FEW;
    if (N > OR_NMAX3) return OR_ST_TOO_MANY;
    double* X = (double*)malloc(sizeof(double) * (size_t)N * p);
    double* W = (double*)malloc(sizeof(double) * (size_t)N * p);
    for (int j = 0; j < N; ++j) {
        or_monomials3(k, dxh[j], dyh[j], dzh[j], X + (size_t)j * p);
        or_abfs3(o->rbf, o->sigma, k, dxh[j], dyh[j], dzh[j], W + (size_t)j * p);
    }
    double M[OR_MAXP * OR_MAXP];
    for (int m = 0; m < p; ++m)
        for (int nn = 0; nn < p; ++nn) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j) acc += X[(size_t)j * p + m] * W[(size_t)j * p + nn];
            M[m * p + nn] = acc;
        }
    or_lu F;
    if (or_lu_factor(&F, M, p) != 0) {
        free(X);
        free(W);
        return OR_ST_SINGULAR;
    }
    double worst = 0.0;
    int maxit = 0;
    for (int d = 0; d < nops; ++d) {
        double C[OR_MAXP], Psi[OR_MAXP], r[OR_MAXP];
        int l;
        or_target3(list[d], p, C, &l);
        double* w = what + (size_t)d * N;
        or_lu_solve(&F, C, Psi);
        for (int j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int nn = 0; nn < p; ++nn) acc += W[(size_t)j * p + nn] * Psi[nn];
            w[j] = acc;
        }
        int it = 0;
        double res = 0.0;
        for (;;) {
            res = 0.0;
            for (int m = 0; m < p; ++m) {
                double acc = 0.0;
                for (int j = 0; j < N; ++j) acc += X[(size_t)j * p + m] * w[j];
                r[m] = C[m] - acc;
                res = fmax(res, fabs(r[m]));
            }
            if (!(res > o->tol_stop) || it >= o->max_iters) break;
            double dPsi[OR_MAXP];
            or_lu_solve(&F, r, dPsi);
            for (int j = 0; j < N; ++j) {
                double acc = 0.0;
                for (int nn = 0; nn < p; ++nn) acc += W[(size_t)j * p + nn] * dPsi[nn];
                w[j] += acc;
            }
            ++it;
        }
        if (!isfinite(res)) res = INFINITY;
        worst = fmax(worst, res);
        if (it > maxit) maxit = it;
    }
    free(X);
    free(W);
    *resid = worst;
    *iters = maxit;
    return (worst <= 1e-10) ? OR_ST_OK : OR_ST_NOT_CONVERGED;
}

int or_weights3(int64_t n, const double* x, const double* y, const double* z, const or_domain3* dom,
                const double* R, int k, const int64_t* row_ptr, const int32_t* col, const or_wopts* o,
                double* w, int8_t* status, double* resid, int8_t* iters) {
    unsigned list[6];
    int nops = or_ops3(o->ops, list);
    int64_t nnz = row_ptr[n];
    double L[3] = {dom->hi[0] - dom->lo[0], dom->hi[1] - dom->lo[1], dom->hi[2] - dom->lo[2]};
    int nbad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nbad)
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = row_ptr[i];
        int N = (int)(row_ptr[i + 1] - s);
        double h = 0.5 * R[i];
        size_t sz = sizeof(double) * (size_t)(N > 0 ? N : 1);
        double *dxh = malloc(sz), *dyh = malloc(sz), *dzh = malloc(sz), *wh = malloc(sz * (size_t)nops);
        for (int j = 0; j < N; ++j) {
            int32_t c = col[s + j];
            dxh[j] = or_wrap(x[c] - x[i], L[0], dom->periodic[0]) / h;
            dyh[j] = or_wrap(y[c] - y[i], L[1], dom->periodic[1]) / h;
            dzh[j] = or_wrap(z[c] - z[i], L[2], dom->periodic[2]) / h;
        }
        double res;
        int it;
        int st = node_weights3(k, N, dxh, dyh, dzh, o, wh, &res, &it);
        for (int d = 0; d < nops; ++d) {
            double hl = (list[d] == OR_OP_LAP) ? h * h : h;
            for (int j = 0; j < N; ++j)
                w[(size_t)d * nnz + s + j] =
                    (st == OR_ST_OK || st == OR_ST_NOT_CONVERGED) ? wh[(size_t)d * N + j] / hl : 0.0;
        }
        status[i] = (int8_t)st;
        resid[i] = res;
        iters[i] = (int8_t)it;
        if (st != OR_ST_OK) nbad++;
        free(dxh);
        free(dyh);
        free(dzh);
        free(wh);
    }
    return nbad;
}

int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_num_threads(int t) { omp_set_num_threads(t); }
