// Reference-element operators (host, FP64).
//
// Sec. II-A: fields are expanded in Lagrange polynomials on N_p nodes
// (text before eq. (10)); the generalized Vandermonde matrices V(j,i) =
// phi_i(r_j) and V_I(q,i) = phi_i(r_q) of the orthonormal basis phi_i give
// V_q = V_I V^{-1} (eq. (20)), M^{-1} = V V^T and P_q = M^{-1} V_q^T W
// (eq. (21)).  Stiffness-type derivative matrices D_u = V_u V^{-1} and the lift
// M^{-1} F of the face-mass matrix of eq. (17) complete the curl operator of
// eqs. (15)-(16).
//
// Orthonormal basis: the Proriol-Koornwinder-Dubiner polynomials in collapsed
// coordinates a = 2(1+r)/(-s-t) - 1, b = 2(1+s)/(1-t) - 1, c = t:
//   phi_ijk = 2 sqrt(2) P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i
//             P_k^{(2i+2j+2,0)}(c) (1-c)^{i+j},
// with orthonormal Jacobi polynomials P_n^{(alpha,beta)}.  Their gradient is
// obtained by the chain rule through (a, b, c); every negative power of
// (1-b) or (1-c) cancels against a factor of the same mode, so the formulas
// below are regular at the collapsed edge and vertex.
#include <cmath>
#include <cstring>

#include "host.hpp"

namespace wdg {

namespace {

// Orthonormal Jacobi polynomial on [-1,1] for the weight (1-x)^al (1+x)^be,
// by the three-term recurrence of the orthonormal family.
double jacobi(int n, double al, double be, double x) {
    const double g0 = std::pow(2.0, al + be + 1.0) / (al + be + 1.0) * std::tgamma(al + 1.0) *
                      std::tgamma(be + 1.0) / std::tgamma(al + be + 1.0);
    double pm = 1.0 / std::sqrt(g0);
    if (n == 0) return pm;
    const double g1 = (al + 1.0) * (be + 1.0) / (al + be + 3.0) * g0;
    double p = ((al + be + 2.0) * x / 2.0 + (al - be) / 2.0) / std::sqrt(g1);
    double a_prev = 2.0 / (2.0 + al + be) * std::sqrt((al + 1.0) * (be + 1.0) / (al + be + 3.0));
    for (int i = 1; i < n; ++i) {
        const double h = 2.0 * i + al + be;
        const double a_next = 2.0 / (h + 2.0) *
                              std::sqrt((i + 1.0) * (i + 1.0 + al + be) * (i + 1.0 + al) * (i + 1.0 + be) /
                                        ((h + 1.0) * (h + 3.0)));
        const double b_i = -(al * al - be * be) / (h * (h + 2.0));
        const double pn = (-a_prev * pm + (x - b_i) * p) / a_next;
        pm = p;
        p = pn;
        a_prev = a_next;
    }
    return p;
}

double djacobi(int n, double al, double be, double x) {
    if (n == 0) return 0.0;
    return std::sqrt(n * (n + al + be + 1.0)) * jacobi(n - 1, al + 1.0, be + 1.0, x);
}

void collapse3(double r, double s, double t, double& a, double& b, double& c) {
    a = (std::fabs(s + t) > 1e-13) ? 2.0 * (1.0 + r) / (-s - t) - 1.0 : -1.0;
    b = (std::fabs(1.0 - t) > 1e-13) ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
    c = t;
}

inline double ipow(double x, int e) {
    double v = 1.0;
    for (int i = 0; i < e; ++i) v *= x;
    return v;
}

// Values and gradients of all modes at one point; grad may be null.
// With gb = 1-b, gc = 1-c: da/dr = 4/(gb gc), da/ds = da/dt = 2(1+a)/(gb gc),
// db/ds = 2/gc, db/dt = (1+b)/gc, dc/dt = 1.
void basis3(int N, double r, double s, double t, double* val, double* gr, double* gs, double* gt) {
    double a, b, c;
    collapse3(r, s, t, a, b, c);
    const double gb = 1.0 - b, gc = 1.0 - c;
    const double norm = 2.0 * std::sqrt(2.0);
    int m = 0;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j)
            for (int k = 0; k <= N - i - j; ++k, ++m) {
                const double A = jacobi(i, 0.0, 0.0, a);
                const double Pj = jacobi(j, 2.0 * i + 1.0, 0.0, b);
                const double Pk = jacobi(k, 2.0 * i + 2.0 * j + 2.0, 0.0, c);
                const double Bt = Pj * ipow(gb, i);
                const double Ct = Pk * ipow(gc, i + j);
                val[m] = norm * A * Bt * Ct;
                if (!gr) continue;
                const double dA = djacobi(i, 0.0, 0.0, a);
                const double dPj = djacobi(j, 2.0 * i + 1.0, 0.0, b);
                const double dPk = djacobi(k, 2.0 * i + 2.0 * j + 2.0, 0.0, c);
                // A' P_j gb^{i-1} P_k gc^{i+j-1}, present only for i >= 1
                const double Ta = (i >= 1) ? dA * Pj * ipow(gb, i - 1) * Pk * ipow(gc, i + j - 1) : 0.0;
                const double dBt = dPj * ipow(gb, i) - ((i >= 1) ? i * Pj * ipow(gb, i - 1) : 0.0);
                // A Bt' P_k gc^{i+j-1}; Bt' = 0 when i + j = 0
                const double Tb = (i + j >= 1) ? A * dBt * Pk * ipow(gc, i + j - 1) : 0.0;
                const double dCt = dPk * ipow(gc, i + j) - ((i + j >= 1) ? (i + j) * Pk * ipow(gc, i + j - 1) : 0.0);
                gr[m] = norm * 4.0 * Ta;
                gs[m] = norm * (2.0 * (1.0 + a) * Ta + 2.0 * Tb);
                gt[m] = norm * (2.0 * (1.0 + a) * Ta + (1.0 + b) * Tb + A * Bt * dCt);
            }
}

// Orthonormal basis on the triangle (-1,-1), (1,-1), (-1,1) (area 2).
void basis2(int N, double r, double s, double* val) {
    const double a = (std::fabs(1.0 - s) > 1e-13) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
    const double b = s;
    int m = 0;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N - i; ++j, ++m)
            val[m] = std::sqrt(2.0) * jacobi(i, 0.0, 0.0, a) * jacobi(j, 2.0 * i + 1.0, 0.0, b) * ipow(1.0 - b, i);
}

}  // namespace

void ortho_basis(int N, double r, double s, double t, double* out) { basis3(N, r, s, t, out, nullptr, nullptr, nullptr); }

Mat matmul(const Mat& A, const Mat& B, int n, int k, int m) {
    Mat C(static_cast<size_t>(n) * m, 0.0);
    for (int i = 0; i < n; ++i)
        for (int l = 0; l < k; ++l) {
            const double a = A[static_cast<size_t>(i) * k + l];
            for (int j = 0; j < m; ++j) C[static_cast<size_t>(i) * m + j] += a * B[static_cast<size_t>(l) * m + j];
        }
    return C;
}

Mat transpose(const Mat& A, int n, int m) {
    Mat T(static_cast<size_t>(n) * m);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) T[static_cast<size_t>(j) * n + i] = A[static_cast<size_t>(i) * m + j];
    return T;
}

// Gauss-Jordan elimination with partial pivoting.
Mat invert(const Mat& A0, int n) {
    Mat A = A0;
    Mat X(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) X[static_cast<size_t>(i) * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[static_cast<size_t>(r) * n + col]) > std::fabs(A[static_cast<size_t>(piv) * n + col])) piv = r;
        if (std::fabs(A[static_cast<size_t>(piv) * n + col]) < 1e-300) throw Error(-1, "singular matrix");
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                std::swap(A[static_cast<size_t>(piv) * n + j], A[static_cast<size_t>(col) * n + j]);
                std::swap(X[static_cast<size_t>(piv) * n + j], X[static_cast<size_t>(col) * n + j]);
            }
        const double d = A[static_cast<size_t>(col) * n + col];
        for (int j = 0; j < n; ++j) {
            A[static_cast<size_t>(col) * n + j] /= d;
            X[static_cast<size_t>(col) * n + j] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[static_cast<size_t>(r) * n + col];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[static_cast<size_t>(r) * n + j] -= f * A[static_cast<size_t>(col) * n + j];
                X[static_cast<size_t>(r) * n + j] -= f * X[static_cast<size_t>(col) * n + j];
            }
        }
    }
    return X;
}

RefElement build_reference(int N, int nq, const double* rst, const double* w) {
    if (N < 1 || N > 4) throw Error(-1, "order N must be 1..4");
    RefElement R;
    R.N = N;
    R.Np = (N + 1) * (N + 2) * (N + 3) / 6;
    R.Nfp = (N + 1) * (N + 2) / 2;
    const int Np = R.Np, Nfp = R.Nfp;
    // Equispaced lattice nodes: c outer, b middle, a inner.
    for (int c = 0; c <= N; ++c)
        for (int b = 0; b <= N - c; ++b)
            for (int a = 0; a <= N - b - c; ++a) {
                R.r.push_back(-1.0 + 2.0 * a / N);
                R.s.push_back(-1.0 + 2.0 * b / N);
                R.t.push_back(-1.0 + 2.0 * c / N);
            }
    // Face node lists (f0: t=-1, f1: s=-1, f2: r+s+t=-1, f3: r=-1), increasing node index.
    R.fmask.assign(4 * Nfp, 0);
    int cnt[4] = {0, 0, 0, 0};
    for (int i = 0; i < Np; ++i) {
        const bool on[4] = {std::fabs(R.t[i] + 1.0) < 1e-12, std::fabs(R.s[i] + 1.0) < 1e-12,
                            std::fabs(R.r[i] + R.s[i] + R.t[i] + 1.0) < 1e-12, std::fabs(R.r[i] + 1.0) < 1e-12};
        for (int f = 0; f < 4; ++f)
            if (on[f]) {
                if (cnt[f] >= Nfp) throw Error(-1, "face node count");
                R.fmask[f * Nfp + cnt[f]++] = i;
            }
    }
    for (int f = 0; f < 4; ++f)
        if (cnt[f] != Nfp) throw Error(-1, "face node count");

    // Vandermonde and gradient Vandermondes.
    R.V.assign(static_cast<size_t>(Np) * Np, 0.0);
    Mat Vr(R.V.size()), Vs(R.V.size()), Vt(R.V.size());
    for (int i = 0; i < Np; ++i)
        basis3(N, R.r[i], R.s[i], R.t[i], &R.V[static_cast<size_t>(i) * Np], &Vr[static_cast<size_t>(i) * Np],
               &Vs[static_cast<size_t>(i) * Np], &Vt[static_cast<size_t>(i) * Np]);
    R.Vinv = invert(R.V, Np);
    R.Minv = matmul(R.V, transpose(R.V, Np, Np), Np, Np, Np);      // M^{-1} = V V^T
    R.M = matmul(transpose(R.Vinv, Np, Np), R.Vinv, Np, Np, Np);    // M = V^{-T} V^{-1}
    R.Dr = matmul(Vr, R.Vinv, Np, Np, Np);
    R.Ds = matmul(Vs, R.Vinv, Np, Np, Np);
    R.Dt = matmul(Vt, R.Vinv, Np, Np, Np);

    // Face mass matrices from the 2D orthonormal basis: M_f = (V_2 V_2^T)^{-1},
    // with face coordinates f0:(r,s), f1:(r,t), f2:(s,t), f3:(s,t).
    Mat E(static_cast<size_t>(Np) * 4 * Nfp, 0.0);
    for (int f = 0; f < 4; ++f) {
        Mat V2(static_cast<size_t>(Nfp) * Nfp);
        for (int m = 0; m < Nfp; ++m) {
            const int n = R.fmask[f * Nfp + m];
            double x = 0, y = 0;
            if (f == 0) { x = R.r[n]; y = R.s[n]; }
            else if (f == 1) { x = R.r[n]; y = R.t[n]; }
            else { x = R.s[n]; y = R.t[n]; }
            basis2(N, x, y, &V2[static_cast<size_t>(m) * Nfp]);
        }
        Mat Mf = invert(matmul(V2, transpose(V2, Nfp, Nfp), Nfp, Nfp, Nfp), Nfp);
        for (int m = 0; m < Nfp; ++m)
            for (int m2 = 0; m2 < Nfp; ++m2)
                E[static_cast<size_t>(R.fmask[f * Nfp + m]) * 4 * Nfp + f * Nfp + m2] = Mf[static_cast<size_t>(m) * Nfp + m2];
    }
    R.LIFT = matmul(R.Minv, E, Np, Np, 4 * Nfp);

    // Cubature: V_q = V_I V^{-1}, P_q = M^{-1} V_q^T W.
    if (nq < 1 || !rst || !w) throw Error(-1, "cubature rule required");
    R.Nq = nq;
    Mat VI(static_cast<size_t>(nq) * Np);
    for (int q = 0; q < nq; ++q) {
        R.rq.push_back(rst[3 * q]);
        R.sq.push_back(rst[3 * q + 1]);
        R.tq.push_back(rst[3 * q + 2]);
        R.wq.push_back(w[q]);
        basis3(N, rst[3 * q], rst[3 * q + 1], rst[3 * q + 2], &VI[static_cast<size_t>(q) * Np], nullptr, nullptr, nullptr);
    }
    R.Vq = matmul(VI, R.Vinv, nq, Np, Np);
    Mat VqTW = transpose(R.Vq, nq, Np);  // [Np][nq]
    for (int i = 0; i < Np; ++i)
        for (int q = 0; q < nq; ++q) VqTW[static_cast<size_t>(i) * nq + q] *= w[q];
    R.Pq = matmul(R.Minv, VqTW, Np, Np, nq);
    // The weight-adjusted inverse needs P_q V_q = I, i.e. a rule exact to degree 2N.
    Mat PV = matmul(R.Pq, R.Vq, Np, nq, Np);
    for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Np; ++j)
            if (std::fabs(PV[static_cast<size_t>(i) * Np + j] - (i == j ? 1.0 : 0.0)) > 1e-9)
                throw Error(-1, "cubature rule is not exact to degree 2N (P_q V_q != I)");
    return R;
}

}  // namespace wdg
