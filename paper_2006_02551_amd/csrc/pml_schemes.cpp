// PML schemes other than the weight-adjusted one, for comparison (C ABI part):
// the direct scheme with stored per-element matrices (eqs. (10)-(15) with the
// weighted mass matrices integrated exactly, the implementation Table I
// measures against) and element-constant coefficients (Sec. III,
// configuration (i)).
//
// Direct scheme, per PML element and axis u.  With W^alpha(i, j) =
// sum_r w_r alpha(x_r) l_i(r_r) l_j(r_r) over the rule points r_r mapped to
// the element (so that M^alpha = J_k W^alpha and M_k = J_k M), the stage
// needs
//   d/dt f_u = (M^a)^-1 [M_k R_u - M^b f_u - M^c P_u],
//   d/dt P_u = M_k^-1 [M^{1/kappa} f_u - M^d P_u],
// and J_k cancels in every product:
//   G_1 = (W^a)^-1 M, G_2 = (W^a)^-1 W^b, G_3 = (W^a)^-1 W^c,
//   G_4 = M^-1 W^{1/kappa}, G_5 = M^-1 W^d.
// The 15 weighted matrices of an element are one product of the
// element-independent table l_i l_j (i <= j) at the rule points with the
// element's 15 weight columns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "context.hpp"

using namespace wdg;

namespace {

// eq. (9) per axis u at one point: out[m][u] for m = a, b, c, d, 1/kappa.
void tensor_entries(const double* sg, const double* kp, double out[5][3]) {
    for (int u = 0; u < 3; ++u) {
        const int v = (u + 1) % 3, w = (u + 2) % 3;
        const double a = kp[v] * kp[w] / kp[u];
        const double b = (sg[v] * kp[w] + sg[w] * kp[v] - a * sg[u]) / kp[u];
        out[0][u] = a;
        out[1][u] = b;
        out[2][u] = sg[v] * sg[w] - b * sg[u];
        out[3][u] = sg[u] / kp[u];
        out[4][u] = 1.0 / kp[u];
    }
}

void profile_at(const PmlParams& pml, const double* x, double* sg, double* kp) {
    for (int d = 0; d < 3; ++d) {
        const double ratio = profile_ratio(x[d], pml.lo[d], pml.hi[d], pml.L[d], pml.order);
        sg[d] = pml.sigma_max[d] * ratio;
        kp[d] = 1.0 + (pml.kappa_max - 1.0) * ratio;
    }
}

template <typename real>
void store(std::vector<unsigned char>& buf, size_t word, double v) {
    reinterpret_cast<real*>(buf.data())[word] = static_cast<real>(v);
}

struct DirectTables {
    int Np = 0, nr = 0, npair = 0;
    std::vector<double> pair;   // [npair][nr]  l_i l_j at the rule points, i <= j
    std::vector<int> pi, pj;    // pair -> (i, j)
    std::vector<double> rw;     // rule weights
    std::vector<double> rr;     // rule points [nr][3]
};

// Products G_1..G_5 for one element (user index k) into out[3][5][Np][Np].
void direct_element(const Setup& S, const DirectTables& T, int k, std::vector<double>& omega, std::vector<double>& W,
                    std::vector<double>& out) {
    const int Np = T.Np, nr = T.nr;
    const int* ev = &S.etov[4 * static_cast<size_t>(k)];
    const double* v0 = &S.vxyz[3 * static_cast<size_t>(ev[0])];
    const double* v1 = &S.vxyz[3 * static_cast<size_t>(ev[1])];
    const double* v2 = &S.vxyz[3 * static_cast<size_t>(ev[2])];
    const double* v3 = &S.vxyz[3 * static_cast<size_t>(ev[3])];
    // weight columns: omega[r][m * 3 + u] = w_r alpha_m,u(x_r)
    for (int r = 0; r < nr; ++r) {
        const double rr = T.rr[3 * r] + 1.0, ss = T.rr[3 * r + 1] + 1.0, tt = T.rr[3 * r + 2] + 1.0;
        double x[3], sg[3], kp[3], al[5][3];
        for (int d = 0; d < 3; ++d) x[d] = v0[d] + 0.5 * ((v1[d] - v0[d]) * rr + (v2[d] - v0[d]) * ss + (v3[d] - v0[d]) * tt);
        profile_at(S.pml, x, sg, kp);
        tensor_entries(sg, kp, al);
        for (int m = 0; m < 5; ++m)
            for (int u = 0; u < 3; ++u) omega[static_cast<size_t>(r) * 16 + m * 3 + u] = T.rw[r] * al[m][u];
    }
    // W[col][i][j] = sum_r l_i l_j omega[r][col]
    for (int pr = 0; pr < T.npair; ++pr) {
        double acc[16] = {0.0};
        const double* pp = &T.pair[static_cast<size_t>(pr) * nr];
        for (int r = 0; r < nr; ++r) {
            const double t = pp[r];
            const double* om = &omega[static_cast<size_t>(r) * 16];
            for (int col = 0; col < 15; ++col) acc[col] += t * om[col];
        }
        const int i = T.pi[pr], j = T.pj[pr];
        for (int col = 0; col < 15; ++col) {
            W[(static_cast<size_t>(col) * Np + i) * Np + j] = acc[col];
            W[(static_cast<size_t>(col) * Np + j) * Np + i] = acc[col];
        }
    }
    const RefElement& R = S.ref;
    const size_t NN = static_cast<size_t>(Np) * Np;
    for (int u = 0; u < 3; ++u) {
        auto Wm = [&](int m) { return Mat(W.begin() + (m * 3 + u) * NN, W.begin() + (m * 3 + u + 1) * NN); };
        const Mat Wainv = invert(Wm(0), Np);
        const Mat G[5] = {matmul(Wainv, R.M, Np, Np, Np), matmul(Wainv, Wm(1), Np, Np, Np), matmul(Wainv, Wm(2), Np, Np, Np),
                          matmul(R.Minv, Wm(4), Np, Np, Np), matmul(R.Minv, Wm(3), Np, Np, Np)};
        for (int m = 0; m < 5; ++m) std::copy(G[m].begin(), G[m].end(), out.begin() + (u * 5 + m) * NN);
    }
}

int build_direct(wdg_ctx* c, int nr, const double* rst, const double* w) {
    const Setup& S = c->S;
    const RefElement& R = S.ref;
    const int Np = R.Np, B = S.B;
    DirectTables T;
    T.Np = Np;
    T.nr = nr;
    T.rw.assign(w, w + nr);
    T.rr.assign(rst, rst + 3 * static_cast<size_t>(nr));
    // Lagrange values at the rule points: l(r) = phi(r)^T V^-1
    std::vector<double> L(static_cast<size_t>(nr) * Np), phi(Np);
    for (int r = 0; r < nr; ++r) {
        ortho_basis(R.N, rst[3 * r], rst[3 * r + 1], rst[3 * r + 2], phi.data());
        for (int i = 0; i < Np; ++i) {
            double v = 0.0;
            for (int n = 0; n < Np; ++n) v += phi[n] * R.Vinv[static_cast<size_t>(n) * Np + i];
            L[static_cast<size_t>(r) * Np + i] = v;
        }
    }
    for (int i = 0; i < Np; ++i)
        for (int j = i; j < Np; ++j) {
            T.pi.push_back(i);
            T.pj.push_back(j);
        }
    T.npair = static_cast<int>(T.pi.size());
    T.pair.resize(static_cast<size_t>(T.npair) * nr);
    for (int pr = 0; pr < T.npair; ++pr)
        for (int r = 0; r < nr; ++r)
            T.pair[static_cast<size_t>(pr) * nr + r] = L[static_cast<size_t>(r) * Np + T.pi[pr]] * L[static_cast<size_t>(r) * Np + T.pj[pr]];

    const size_t NN = static_cast<size_t>(Np) * Np;
    const size_t blk_words = 3 * kDirectMats * NN * B;
    const size_t rs = c->rsize;
    c->pml_mats.alloc(static_cast<size_t>(S.nblk_pml) * blk_words * rs);
    c->pml_work.alloc(static_cast<size_t>(S.nblk_pml) * 6 * Np * B * rs);
    if (S.nblk_pml == 0) return WDG_OK;

    const int nthreads = std::max(1, std::min(16, static_cast<int>(std::thread::hardware_concurrency())));
    // a round computes nthreads runs of `per` blocks on the host, then uploads them in one copy
    const int per = std::max(1, static_cast<int>((64u << 20) / (blk_words * rs)));
    std::vector<unsigned char> host(static_cast<size_t>(nthreads) * per * blk_words * rs);
    for (int b0 = 0; b0 < S.nblk_pml; b0 += nthreads * per) {
        const int b1 = std::min(S.nblk_pml, b0 + nthreads * per);
        std::vector<std::thread> pool;
        std::vector<std::string> errors(nthreads);
        for (int th = 0; th < nthreads; ++th) {
            pool.emplace_back([&, th]() {
                try {
                    std::vector<double> omega(static_cast<size_t>(nr) * 16, 0.0), W(15 * NN), G(15 * NN);
                    const int lo = b0 + th * per, hi = std::min(b1, lo + per);
                    for (int blk = lo; blk < hi; ++blk)
                        for (int lane = 0; lane < B; ++lane) {
                            const int k = S.slot_elem[static_cast<size_t>(blk) * B + lane];
                            if (k >= 0) direct_element(S, T, k, omega, W, G);
                            else std::fill(G.begin(), G.end(), 0.0);
                            const size_t base = static_cast<size_t>(blk - b0) * blk_words + lane;
                            for (size_t e = 0; e < 15 * NN; ++e) {
                                const size_t word = base + e * B;
                                if (rs == 8) store<double>(host, word, G[e]);
                                else store<float>(host, word, G[e]);
                            }
                        }
                } catch (const std::exception& e) {
                    errors[th] = e.what();
                }
            });
        }
        for (auto& t : pool) t.join();
        for (const auto& e : errors)
            if (!e.empty()) throw Error(WDG_EINVAL, "direct-scheme setup: " + e);
        hip_check(hipMemcpy(static_cast<char*>(c->pml_mats.p) + static_cast<size_t>(b0) * blk_words * rs, host.data(),
                            static_cast<size_t>(b1 - b0) * blk_words * rs, hipMemcpyHostToDevice),
                  "upload direct matrices");
    }
    return WDG_OK;
}

int build_constant(wdg_ctx* c) {
    const Setup& S = c->S;
    const int Np = S.ref.Np, B = S.B;
    std::vector<double> v(static_cast<size_t>(S.nblk_pml) * 6 * B, 0.0);
    for (size_t slot = 0; slot < static_cast<size_t>(S.nblk_pml) * B; ++slot) {
        const size_t blk = slot / B, lane = slot % B;
        const int k = S.slot_elem[slot];
        for (int u = 0; u < 3; ++u) {
            double sg = 0.0, kp = 1.0;
            if (k >= 0) {
                // node farthest beyond the interface along u (first one on ties)
                int far = 0;
                double dmax = -1.0;
                for (int i = 0; i < Np; ++i) {
                    const double x = S.xnodes[(static_cast<size_t>(k) * Np + i) * 3 + u];
                    const double d = std::max(0.0, std::max(x - S.pml.hi[u], S.pml.lo[u] - x));
                    if (d > dmax) {
                        dmax = d;
                        far = i;
                    }
                }
                const double x = S.xnodes[(static_cast<size_t>(k) * Np + far) * 3 + u];
                const double ratio = profile_ratio(x, S.pml.lo[u], S.pml.hi[u], S.pml.L[u], S.pml.order);
                sg = S.pml.sigma_max[u] * ratio;
                kp = 1.0 + (S.pml.kappa_max - 1.0) * ratio;
            }
            v[(blk * 6 + u) * B + lane] = sg;
            v[(blk * 6 + 3 + u) * B + lane] = kp;
        }
    }
    const auto bytes = to_real(v, c->precision);
    c->pml_mats.upload(bytes.data(), bytes.size());
    return WDG_OK;
}

}  // namespace

extern "C" {

int32_t wdg_set_pml_scheme(wdg_ctx* c, int32_t scheme, int32_t nr, const double* rst, const double* w) {
    if (!c) return WDG_EINVAL;
    if (scheme != WDG_PML_WAA && scheme != WDG_PML_DIRECT && scheme != WDG_PML_CONSTANT)
        return fail(c, WDG_EINVAL, "unknown PML scheme");
    if (c->host_only) return fail(c, WDG_ESTATE, "host-only context");
    if (scheme == WDG_PML_DIRECT) {
        if (nr < 1 || !rst || !w) return fail(c, WDG_EINVAL, "the direct scheme needs a rule (nr >= 1 points and weights)");
        for (int r = 0; r < nr; ++r)
            if (!std::isfinite(w[r]) || !std::isfinite(rst[3 * r]) || !std::isfinite(rst[3 * r + 1]) ||
                !std::isfinite(rst[3 * r + 2]))
                return fail(c, WDG_EINVAL, "rule points and weights must be finite");
    }
    if (scheme != WDG_PML_WAA && c->sigma_custom)
        return fail(c, WDG_ESTATE,
                    "the direct and element-constant schemes sample the method's profile, but sigma at the cubature "
                    "points was replaced");
    return guarded(c, [&]() -> int {
        c->drop_graph();
        c->pml_mats.alloc(0);
        c->pml_work.alloc(0);
        c->pml_scheme = WDG_PML_WAA;
        int rc = WDG_OK;
        if (scheme == WDG_PML_DIRECT) rc = build_direct(c, nr, rst, w);
        else if (scheme == WDG_PML_CONSTANT) rc = build_constant(c);
        if (rc != WDG_OK) {
            c->pml_mats.alloc(0);
            c->pml_work.alloc(0);
            return rc;
        }
        c->pml_scheme = scheme;
        return WDG_OK;
    });
}

}  // extern "C"
