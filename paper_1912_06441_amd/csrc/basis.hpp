// basis.hpp -- device-side monomials, ABFs and RBF derivatives for gfx950.
//
// Element m of the monomial vector X (Sec. 2 eq. 1 of King, Lind & Nasar)
// is x^a y^b / (a! b!) with (a, b) running over total order n = 1..k and,
// within an order, a = n, ..., 0.  The element order for order k is a prefix
// of the order-8 order, so one table serves every k <= 8.
//
// ABF families (Sec. 3.2, App. A):
//   HERMITE: W_m = H_a(sigma x) H_b(sigma y) phi(|d|)      (physicists' Hermite)
//   PAPER:   W_m = d^a_x d^b_y W0(|d|) for a + b <= 3, and dW0/dr * d^a_x d^b_y |d|
//            for a + b >= 4 (App. A truncation).
//   PAPER_D1: dW0/dr * d^a_x d^b_y |d| for every element.
// The PAPER family is evaluated through s = r^2 / 2: for a radial function
// F(r) = G(s),
//   d^a_x d^b_y G(s) = sum_{i,l} c_{a,i} c_{b,l} x^(2i-a) y^(2l-b) G^(i+l)(s),
//   c_{a,i} = a! / ((2i-a)! (a-i)! 2^(a-i)),  ceil(a/2) <= i <= a,
// with G' = F'/r, G'' = (F'' - F'/r)/r^2, G''' = (F''' - 3F''/r + 3F'/r^2)/r^3,
// and for F = r: G^(m) = (-1)^(m-1) (2m-3)!! r^(1-2m).
#pragma once

#include <hip/hip_runtime.h>

namespace labfm {

constexpr int KMAX = 8;
constexpr int PMAX = 44;
constexpr int NMAX = LABFM_MAX_NEIGHBOURS;
constexpr int MAXOPS = 5;

constexpr int p_of_k(int k) { return (k * k + 3 * k) / 2; }

struct ElemTable {
    int a[PMAX];
    int b[PMAX];
};
constexpr ElemTable make_elems() {
    ElemTable t{};
    int m = 0;
    for (int n = 1; n <= KMAX; ++n)
        for (int a = n; a >= 0; --a) {
            t.a[m] = a;
            t.b[m] = n - a;
            ++m;
        }
    return t;
}
constexpr ElemTable ELEM = make_elems();

constexpr double inv_fact(int a) {
    double f = 1.0;
    for (int i = 2; i <= a; ++i) f *= i;
    return 1.0 / f;
}

// Faa di Bruno table through s = r^2/2: for element (a,b), the terms
// coef * x^ex * y^ey * G^(m)(s).  At most 9 terms per element up to order 8.
struct FdbTerm {
    double coef;
    int ex, ey, m;
};
struct FdbTable {
    FdbTerm t[PMAX][9];
    int nt[PMAX];
};
constexpr double cfac(int a, int i) {
    // a! / ((2i-a)! (a-i)! 2^(a-i))
    double num = 1.0;
    for (int q = 2; q <= a; ++q) num *= q;
    double den = 1.0;
    for (int q = 2; q <= 2 * i - a; ++q) den *= q;
    for (int q = 2; q <= a - i; ++q) den *= q;
    for (int q = 0; q < a - i; ++q) den *= 2.0;
    return num / den;
}
constexpr FdbTable make_fdb() {
    FdbTable T{};
    for (int m = 0; m < PMAX; ++m) {
        int a = ELEM.a[m], b = ELEM.b[m];
        int c = 0;
        for (int i = (a + 1) / 2; i <= a; ++i)
            for (int l = (b + 1) / 2; l <= b; ++l) {
                T.t[m][c].coef = cfac(a, i) * cfac(b, l);
                T.t[m][c].ex = 2 * i - a;
                T.t[m][c].ey = 2 * l - b;
                T.t[m][c].m = i + l;
                ++c;
            }
        T.nt[m] = c;
    }
    return T;
}
constexpr FdbTable FDB = make_fdb();

// (-1)^(m-1) (2m-3)!!  : coefficient of r^(1-2m) in d^m/ds^m of r = sqrt(2 s)
constexpr double rdiff_coef(int m) {
    double v = 1.0;
    for (int q = 1; q <= 2 * m - 3; q += 2) v *= q;
    return (m % 2 == 1) ? v : -v;
}

// RBF value and first three q-derivatives.  Returns F[0..3].
__device__ inline void rbf_eval(int rbf, double q, double* F) {
    const double pi = 3.14159265358979323846;
    if (rbf == LABFM_RBF_GAUSSIAN) {
        double g = (9.0 / pi) * exp(-9.0 * q * q);
        F[0] = g;
        F[1] = -18.0 * q * g;
        F[2] = (324.0 * q * q - 18.0) * g;
        F[3] = (972.0 * q - 5832.0 * q * q * q) * g;
        return;
    }
    if (q >= 2.0) {
        F[0] = F[1] = F[2] = F[3] = 0.0;
        return;
    }
    double t = 1.0 - 0.5 * q;
    if (rbf == LABFM_RBF_WENDLAND_C2) {
        double t2 = t * t, t3 = t2 * t;
        F[0] = t3 * t * (1.0 + 2.0 * q);
        F[1] = -5.0 * q * t3;
        F[2] = 7.5 * q * t2 - 5.0 * t3;
        F[3] = 15.0 * t2 - 7.5 * q * t;
    } else if (rbf == LABFM_RBF_CONE) {
        const double c = 3.0 / (4.0 * pi);
        F[0] = c * t;
        F[1] = -0.5 * c;
        F[2] = 0.0;
        F[3] = 0.0;
    } else if (rbf == LABFM_RBF_QUADRATIC) {
        const double c = 3.0 / (16.0 * pi);
        F[0] = c * (q - 2.0) * (q - 2.0);
        F[1] = 2.0 * c * (q - 2.0);
        F[2] = 2.0 * c;
        F[3] = 0.0;
    } else {  // Wendland C6: c t^8 (4q^3 + 6.25q^2 + 4q + 1)
        const double c = 78.0 / (28.0 * pi);
        double t2 = t * t, t4 = t2 * t2, t5 = t4 * t, t6 = t4 * t2, t7 = t6 * t, t8 = t4 * t4;
        double P0 = ((4.0 * q + 6.25) * q + 4.0) * q + 1.0;
        double P1 = (12.0 * q + 12.5) * q + 4.0;
        double P2 = 24.0 * q + 12.5;
        double P3 = 24.0;
        double T0 = t8, T1 = -4.0 * t7, T2 = 14.0 * t6, T3 = -42.0 * t5;
        F[0] = c * T0 * P0;
        F[1] = c * (T1 * P0 + T0 * P1);
        F[2] = c * (T2 * P0 + 2.0 * T1 * P1 + T0 * P2);
        F[3] = c * (T3 * P0 + 3.0 * T2 * P1 + 3.0 * T1 * P2 + T0 * P3);
    }
}

// Per-offset evaluation state (registers of one lane).
template <int K>
struct BasisState {
    double px[K + 1], py[K + 1];  // powers of the offset components
    double hx[K + 1], hy[K + 1];  // Hermite polynomials (HERMITE) or unused
    double phi;                   // radial factor (HERMITE) or W0'(q) (PAPER)
    double G[4];                  // G^(m)(s), m = 1..3, for the PAPER family
    double ir;                    // 1 / |d| (PAPER)
    bool ok;                      // false if the ABFs are undefined here
};

template <int K, int FAM>
__device__ inline void basis_prepare(BasisState<K>& B, double dx, double dy, int rbf, double sigma) {
    B.px[0] = 1.0;
    B.py[0] = 1.0;
#pragma unroll
    for (int e = 1; e <= K; ++e) {
        B.px[e] = B.px[e - 1] * dx;
        B.py[e] = B.py[e - 1] * dy;
    }
    double q = sqrt(dx * dx + dy * dy);
    double F[4];
    rbf_eval(rbf, q, F);
    B.ok = true;
    if (FAM == LABFM_ABF_HERMITE) {
        double tx = sigma * dx, ty = sigma * dy;
        B.hx[0] = 1.0;
        B.hy[0] = 1.0;
        if (K >= 1) {
            B.hx[1] = 2.0 * tx;
            B.hy[1] = 2.0 * ty;
        }
#pragma unroll
        for (int e = 1; e < K; ++e) {
            B.hx[e + 1] = 2.0 * tx * B.hx[e] - 2.0 * e * B.hx[e - 1];
            B.hy[e + 1] = 2.0 * ty * B.hy[e] - 2.0 * e * B.hy[e - 1];
        }
        B.phi = F[0];
    } else {
        if (!(q > 0.0)) {
            B.ok = false;
            q = 1.0;
        }
        double ir = 1.0 / q;
        // G^(m) for m = 1..3 of W0 (full derivatives, orders <= 3)
        B.G[0] = 0.0;
        B.G[1] = F[1] * ir;
        B.G[2] = (F[2] - F[1] * ir) * ir * ir;
        B.G[3] = (F[3] - 3.0 * F[2] * ir + 3.0 * F[1] * ir * ir) * ir * ir * ir;
        B.phi = F[1];  // W0'(q) for the truncated elements
        B.ir = ir;
    }
}

template <int K>
__device__ inline double monomial(const BasisState<K>& B, int m) {
    int a = ELEM.a[m], b = ELEM.b[m];
    return B.px[a] * B.py[b] * (inv_fact(a) * inv_fact(b));
}

template <int K, int FAM>
__device__ inline double abf(const BasisState<K>& B, int m) {
    int a = ELEM.a[m], b = ELEM.b[m];
    if (FAM == LABFM_ABF_HERMITE) return B.hx[a] * B.hy[b] * B.phi;
    int n = a + b;
    double acc = 0.0;
    if (FAM == LABFM_ABF_PAPER && n <= 3) {
        for (int t = 0; t < FDB.nt[m]; ++t) {
            const FdbTerm& T = FDB.t[m][t];
            acc += T.coef * B.px[T.ex] * B.py[T.ey] * B.G[T.m];
        }
        return acc;
    }
    // dW0/dr * d^a_x d^b_y |d|: orders >= 4 of PAPER, every order of PAPER_D1
    double ir = B.ir;
    for (int t = 0; t < FDB.nt[m]; ++t) {
        const FdbTerm& T = FDB.t[m][t];
        // r^(1 - 2 T.m)
        double rp = 1.0;
        for (int e = 0; e < 2 * T.m - 1; ++e) rp *= ir;
        acc += T.coef * rdiff_coef(T.m) * B.px[T.ex] * B.py[T.ey] * rp;
    }
    return B.phi * acc;
}

}  // namespace labfm
