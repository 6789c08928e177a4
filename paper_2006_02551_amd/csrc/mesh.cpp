// Geometry, connectivity, PML sampling and device ordering (host, FP64).
//
// Sec. II-A, text after eq. (17): on an affine tetrahedron M_k = J_k M, so the
// element enters the curl operator only through its metric terms, outward
// normals and the surface-to-volume ratio Fscale = sJ/J of each face, and
// through its face neighbours k'.  The PML coefficients of eq. (9) are sampled
// at the physical images of the cubature points (eqs. (19)-(20)); only
// sigma_u (and kappa_u when it is not identically one) is stored, 3 (6) words
// per cubature point, instead of the 15 coefficient samples of Sec. II-B.
//
// Construction:
//  * affine map x = v0 + [x_r x_s x_t](r+1, s+1, t+1) with x_r = (v1-v0)/2 ...;
//    grad r = (x_s x x_t)/J, grad s = (x_t x x_r)/J, grad t = (x_r x x_s)/J;
//  * unnormalised outward normals -grad t, -grad s, grad(r+s+t), -grad r for
//    faces t=-1, s=-1, r+s+t=-1, r=-1; Fscale is their length and sJ = Fscale J;
//  * faces are matched by sorting their vertex triples; face nodes are matched
//    exactly through their integer barycentric weights on the shared global
//    vertices, so no coordinate tolerance is involved; an optional vertex
//    identification replaces the vertex numbers in both (periodic meshes: the
//    faces and nodes of a periodic pair meet on identified vertices);
//  * PML elements come first, then interior elements; inside each class the
//    elements are grouped by face-connected component (numbered in order of
//    their lowest element index), ordered along a Morton curve of their
//    centroids within a component, regrouped (within chunks of 1024 elements of
//    that order) into runs of 16 elements grown over shared faces (the element
//    tiles of the matrix-core stage kernel, so that more face neighbours lie in
//    the same tile), and packed into blocks of B element slots.  A single mesh is one component; a batch of disjoint
//    meshes that overlap in space keeps each mesh contiguous, so face
//    neighbours stay close.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "host.hpp"

namespace wdg {

namespace {

inline void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

const int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};

// Regroups an element list (Morton order) into consecutive runs of G elements
// grown over shared faces: a run starts from the unassigned element with the
// most faces on the previous run (else the next unassigned element in list
// order) and repeatedly takes the unassigned face neighbour with the most faces
// on the run, ties going to the earlier list position.  Only elements of the
// list are taken.  Returns the new order.
std::vector<int> grow_runs(const std::vector<int>& order, const std::vector<int>& etoe, int K, int G) {
    const int n = static_cast<int>(order.size());
    std::vector<int> pos(K, -1), cnt(K, 0), front, out;
    std::vector<char> taken(K, 0);
    std::vector<std::pair<int, int>> carry;  // (element, faces on the previous run)
    for (int i = 0; i < n; ++i) pos[order[i]] = i;
    out.reserve(n);
    int next = 0;  // first list position that may still be unassigned
    const int64_t nn = n + 1;
    auto take = [&](int e) {
        taken[e] = 1;
        out.push_back(e);
        for (int f = 0; f < 4; ++f) {
            const int k2 = etoe[4 * static_cast<size_t>(e) + f];
            if (k2 != e && pos[k2] >= 0 && !taken[k2] && cnt[k2]++ == 0) front.push_back(k2);
        }
    };
    auto next_unassigned = [&]() {
        while (taken[order[next]]) ++next;
        return order[next];
    };
    while (static_cast<int>(out.size()) < n) {
        int seed = -1;
        int64_t best = -1;
        for (const auto& ec : carry)
            if (!taken[ec.first] && static_cast<int64_t>(ec.second) * nn - pos[ec.first] > best) {
                best = static_cast<int64_t>(ec.second) * nn - pos[ec.first];
                seed = ec.first;
            }
        front.clear();
        take(seed >= 0 ? seed : next_unassigned());
        for (int m = 1; m < G && static_cast<int>(out.size()) < n; ++m) {
            int pick = -1;
            best = -1;
            for (const int e : front)
                if (!taken[e] && static_cast<int64_t>(cnt[e]) * nn - pos[e] > best) {
                    best = static_cast<int64_t>(cnt[e]) * nn - pos[e];
                    pick = e;
                }
            take(pick >= 0 ? pick : next_unassigned());
        }
        carry.clear();
        for (const int e : front) {
            if (!taken[e]) carry.push_back({e, cnt[e]});
            cnt[e] = 0;
        }
    }
    return out;
}

uint64_t spread3(uint64_t x) {  // 21 bits -> every third bit
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

}  // namespace

double profile_ratio(double x, double lo, double hi, double L, double p) {
    const double d = std::max(0.0, std::max(x - hi, lo - x));
    if (d <= 0.0) return 0.0;
    return std::pow(d / L, p);
}

Setup build_setup(int nv, const double* vxyz, int K, const int* etov_in, const int* vertex_id, int N, int nq,
                  const double* rst, const double* w, const PmlParams& pml, double flux_alpha, bool align_components) {
    if (K <= 0 || nv <= 0 || !vxyz || !etov_in) throw Error(-2, "empty mesh");
    if (vertex_id)
        for (int i = 0; i < nv; ++i)
            if (vertex_id[i] < 0 || vertex_id[i] >= nv) throw Error(-2, "vertex identification out of range");
    auto vid = [&](int v) { return vertex_id ? vertex_id[v] : v; };
    Setup S;
    S.ref = build_reference(N, nq, rst, w);
    const RefElement& R = S.ref;
    const int Np = R.Np, Nfp = R.Nfp, Nq = R.Nq;
    S.K = K;
    S.flux_alpha = flux_alpha;
    S.vxyz.assign(vxyz, vxyz + 3 * static_cast<size_t>(nv));
    S.etov.assign(etov_in, etov_in + 4 * static_cast<size_t>(K));
    S.J.resize(K);
    S.metric.resize(9 * static_cast<size_t>(K));
    S.nrm.resize(12 * static_cast<size_t>(K));
    S.Fscale.resize(4 * static_cast<size_t>(K));
    S.xnodes.resize(static_cast<size_t>(K) * Np * 3);
    double fsmax = 0.0;
    for (int k = 0; k < K; ++k) {
        int* ev = &S.etov[4 * static_cast<size_t>(k)];
        for (int i = 0; i < 4; ++i)
            if (ev[i] < 0 || ev[i] >= nv) throw Error(-2, "vertex index out of range");
        const double* v[4];
        for (int i = 0; i < 4; ++i) v[i] = &S.vxyz[3 * static_cast<size_t>(ev[i])];
        double e1[3], e2[3], e3[3], c23[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = v[1][d] - v[0][d];
            e2[d] = v[2][d] - v[0][d];
            e3[d] = v[3][d] - v[0][d];
        }
        cross3(e2, e3, c23);
        double det6 = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
        if (det6 < 0) {
            std::swap(ev[2], ev[3]);
            std::swap(v[2], v[3]);
            for (int d = 0; d < 3; ++d) std::swap(e2[d], e3[d]);
            det6 = -det6;
        }
        double scale = 0.0;
        for (int d = 0; d < 3; ++d) scale = std::max({scale, std::fabs(e1[d]), std::fabs(e2[d]), std::fabs(e3[d])});
        if (!(det6 > 1e-12 * scale * scale * scale)) throw Error(-2, "degenerate tetrahedron");
        double xr[3], xs[3], xt[3];
        for (int d = 0; d < 3; ++d) {
            xr[d] = 0.5 * e1[d];
            xs[d] = 0.5 * e2[d];
            xt[d] = 0.5 * e3[d];
        }
        double gr[3], gs[3], gt[3];
        cross3(xs, xt, gr);
        cross3(xt, xr, gs);
        cross3(xr, xs, gt);
        const double J = xr[0] * gr[0] + xr[1] * gr[1] + xr[2] * gr[2];
        for (int d = 0; d < 3; ++d) {
            gr[d] /= J;
            gs[d] /= J;
            gt[d] /= J;
        }
        S.J[k] = J;
        double* mt = &S.metric[9 * static_cast<size_t>(k)];
        for (int d = 0; d < 3; ++d) {
            mt[d] = gr[d];
            mt[3 + d] = gs[d];
            mt[6 + d] = gt[d];
        }
        double raw[4][3];
        for (int d = 0; d < 3; ++d) {
            raw[0][d] = -gt[d];
            raw[1][d] = -gs[d];
            raw[2][d] = gr[d] + gs[d] + gt[d];
            raw[3][d] = -gr[d];
        }
        for (int f = 0; f < 4; ++f) {
            const double len = std::sqrt(raw[f][0] * raw[f][0] + raw[f][1] * raw[f][1] + raw[f][2] * raw[f][2]);
            for (int d = 0; d < 3; ++d) S.nrm[12 * static_cast<size_t>(k) + 3 * f + d] = raw[f][d] / len;
            S.Fscale[4 * static_cast<size_t>(k) + f] = len;
            fsmax = std::max(fsmax, len);
        }
        for (int i = 0; i < Np; ++i)
            for (int d = 0; d < 3; ++d)
                S.xnodes[(static_cast<size_t>(k) * Np + i) * 3 + d] =
                    v[0][d] + xr[d] * (R.r[i] + 1.0) + xs[d] * (R.s[i] + 1.0) + xt[d] * (R.t[i] + 1.0);
    }
    S.dt_unit = 1.0 / ((N + 1.0) * (N + 1.0) * fsmax);

    // ---- face matching by sorted (identified) vertex triples
    for (int k = 0; k < K; ++k) {
        const int* ev = &S.etov[4 * static_cast<size_t>(k)];
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j)
                if (vid(ev[i]) == vid(ev[j])) throw Error(-2, "the vertex identification collapses an element");
    }
    struct FaceRec {
        std::array<int, 3> key;
        int k, f;
    };
    std::vector<FaceRec> faces;
    faces.reserve(4 * static_cast<size_t>(K));
    for (int k = 0; k < K; ++k)
        for (int f = 0; f < 4; ++f) {
            std::array<int, 3> key;
            for (int i = 0; i < 3; ++i) key[i] = vid(S.etov[4 * static_cast<size_t>(k) + kFaceVerts[f][i]]);
            std::sort(key.begin(), key.end());
            faces.push_back({key, k, f});
        }
    std::sort(faces.begin(), faces.end(), [](const FaceRec& a, const FaceRec& b) {
        if (a.key != b.key) return a.key < b.key;
        if (a.k != b.k) return a.k < b.k;
        return a.f < b.f;
    });
    S.etoe.resize(4 * static_cast<size_t>(K));
    S.etof.resize(4 * static_cast<size_t>(K));
    for (int k = 0; k < K; ++k)
        for (int f = 0; f < 4; ++f) {
            S.etoe[4 * static_cast<size_t>(k) + f] = k;
            S.etof[4 * static_cast<size_t>(k) + f] = f;
        }
    for (size_t i = 0; i < faces.size();) {
        size_t j = i;
        while (j < faces.size() && faces[j].key == faces[i].key) ++j;
        if (j - i > 2) throw Error(-2, "non-manifold face");
        if (j - i == 2) {
            const FaceRec& a = faces[i];
            const FaceRec& b = faces[i + 1];
            if (a.k == b.k) throw Error(-2, "element with repeated face");
            S.etoe[4 * static_cast<size_t>(a.k) + a.f] = b.k;
            S.etof[4 * static_cast<size_t>(a.k) + a.f] = b.f;
            S.etoe[4 * static_cast<size_t>(b.k) + b.f] = a.k;
            S.etof[4 * static_cast<size_t>(b.k) + b.f] = a.f;
        }
        i = j;
    }

    // ---- face-node matching through integer barycentric weights.
    // Node i has lattice weights (N-a-b-c, a, b, c) on the element's vertices v0..v3.
    std::vector<std::array<int, 4>> lam(Np);
    for (int i = 0; i < Np; ++i) {
        const int a = static_cast<int>(std::lround((R.r[i] + 1.0) * N / 2.0));
        const int b = static_cast<int>(std::lround((R.s[i] + 1.0) * N / 2.0));
        const int c = static_cast<int>(std::lround((R.t[i] + 1.0) * N / 2.0));
        lam[i] = {N - a - b - c, a, b, c};
    }
    auto node_key = [&](int k, int node) {
        // sorted (global vertex, weight) pairs over the vertices with nonzero weight
        std::array<std::pair<int, int>, 4> kv;
        int n = 0;
        for (int v = 0; v < 4; ++v)
            if (lam[node][v] != 0) kv[n++] = {vid(S.etov[4 * static_cast<size_t>(k) + v]), lam[node][v]};
        std::sort(kv.begin(), kv.begin() + n);
        std::array<int, 8> key;
        key.fill(-1);
        for (int i = 0; i < n; ++i) {
            key[2 * i] = kv[i].first;
            key[2 * i + 1] = kv[i].second;
        }
        return key;
    };
    S.nbr_node.resize(static_cast<size_t>(K) * 4 * Nfp);
    for (int k = 0; k < K; ++k)
        for (int f = 0; f < 4; ++f) {
            const int k2 = S.etoe[4 * static_cast<size_t>(k) + f];
            const int f2 = S.etof[4 * static_cast<size_t>(k) + f];
            for (int m = 0; m < Nfp; ++m) {
                const int node = R.fmask[f * Nfp + m];
                int found = node;
                if (k2 != k) {
                    const auto key = node_key(k, node);
                    found = -1;
                    for (int m2 = 0; m2 < Nfp; ++m2) {
                        const int n2 = R.fmask[f2 * Nfp + m2];
                        if (node_key(k2, n2) == key) {
                            found = n2;
                            break;
                        }
                    }
                    if (found < 0) throw Error(-2, "face nodes do not match (non-conforming face)");
                }
                S.nbr_node[(static_cast<size_t>(k) * 4 + f) * Nfp + m] = found;
            }
        }

    // ---- PML sampling at physical cubature points
    S.sigma.assign(static_cast<size_t>(K) * Nq * 3, 0.0);
    S.kappa.assign(static_cast<size_t>(K) * Nq * 3, 1.0);
    S.is_pml.assign(K, 0);
    S.has_kappa = pml.kappa_max != 1.0;
    S.xq.assign(static_cast<size_t>(K) * Nq * 3, 0.0);
    S.pml = pml;
    for (int k = 0; k < K; ++k) {
        const int* ev = &S.etov[4 * static_cast<size_t>(k)];
        const double* v0 = &S.vxyz[3 * static_cast<size_t>(ev[0])];
        const double* v1 = &S.vxyz[3 * static_cast<size_t>(ev[1])];
        const double* v2 = &S.vxyz[3 * static_cast<size_t>(ev[2])];
        const double* v3 = &S.vxyz[3 * static_cast<size_t>(ev[3])];
        bool any = false;
        for (int q = 0; q < Nq; ++q) {
            const double rr = R.rq[q] + 1.0, ss = R.sq[q] + 1.0, tt = R.tq[q] + 1.0;
            for (int d = 0; d < 3; ++d) {
                const double x = v0[d] + 0.5 * ((v1[d] - v0[d]) * rr + (v2[d] - v0[d]) * ss + (v3[d] - v0[d]) * tt);
                S.xq[(static_cast<size_t>(k) * Nq + q) * 3 + d] = x;
                const double ratio = profile_ratio(x, pml.lo[d], pml.hi[d], pml.L[d], pml.order);
                const double sg = pml.sigma_max[d] * ratio;
                const double kp = 1.0 + (pml.kappa_max - 1.0) * ratio;
                S.sigma[(static_cast<size_t>(k) * Nq + q) * 3 + d] = sg;
                S.kappa[(static_cast<size_t>(k) * Nq + q) * 3 + d] = kp;
                if (sg != 0.0 || kp != 1.0) any = true;
            }
        }
        S.is_pml[k] = any ? 1 : 0;
    }

    // ---- ordering: PML class first, then component, then Morton order of centroids, regrouped
    // into face-grown runs of 16 within chunks of the curve
    std::vector<int> comp(K, -1);
    {
        std::vector<int> stack;
        int ncomp = 0;
        for (int k0 = 0; k0 < K; ++k0) {
            if (comp[k0] >= 0) continue;
            comp[k0] = ncomp;
            stack.assign(1, k0);
            while (!stack.empty()) {
                const int k = stack.back();
                stack.pop_back();
                for (int f = 0; f < 4; ++f) {
                    const int k2 = S.etoe[4 * static_cast<size_t>(k) + f];
                    if (comp[k2] < 0) {
                        comp[k2] = ncomp;
                        stack.push_back(k2);
                    }
                }
            }
            ++ncomp;
        }
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < nv; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], vxyz[3 * i + d]);
            hi[d] = std::max(hi[d], vxyz[3 * i + d]);
        }
    std::vector<std::pair<std::pair<int, uint64_t>, int>> pml_list, int_list;
    for (int k = 0; k < K; ++k) {
        uint64_t code = 0;
        for (int d = 0; d < 3; ++d) {
            double c = 0;
            for (int i = 0; i < 4; ++i) c += 0.25 * S.vxyz[3 * static_cast<size_t>(S.etov[4 * static_cast<size_t>(k) + i]) + d];
            const double u = (hi[d] > lo[d]) ? (c - lo[d]) / (hi[d] - lo[d]) : 0.0;
            const uint64_t iu = static_cast<uint64_t>(std::min(std::max(u, 0.0), 1.0) * 2097151.0);
            code |= spread3(iu) << d;
        }
        (S.is_pml[k] ? pml_list : int_list).push_back({{comp[k], code}, k});
    }
    std::sort(pml_list.begin(), pml_list.end());
    std::sort(int_list.begin(), int_list.end());
    std::vector<int> pml_order, int_order;
    for (const auto& x : pml_list) pml_order.push_back(x.second);
    for (const auto& x : int_list) int_order.push_back(x.second);
    // Runs are grown within consecutive chunks of 1024 elements of the Morton order: the chunks keep
    // the curve's large-scale locality (what the L2 caches see across concurrent workgroups; runs
    // grown over the whole class wander and raised the stage kernel's HBM reads by a fifth).  With
    // aligned components the chunks restart at every component.
    constexpr size_t kChunk = 1024;
    S.ncomp = 1 + *std::max_element(comp.begin(), comp.end());
    S.comp = comp;
    S.aligned = align_components;
    for (auto* ord : {&pml_order, &int_order}) {
        std::vector<int> out;
        out.reserve(ord->size());
        size_t i = 0;
        while (i < ord->size()) {
            size_t end = std::min(ord->size(), i + kChunk);
            if (align_components)
                for (size_t e = i + 1; e < end; ++e)
                    if (comp[(*ord)[e]] != comp[(*ord)[i]]) {
                        end = e;
                        break;
                    }
            const std::vector<int> part(ord->begin() + i, ord->begin() + end);
            const std::vector<int> grown = grow_runs(part, S.etoe, K, 16);
            out.insert(out.end(), grown.begin(), grown.end());
            i = end;
        }
        *ord = out;
    }
    S.K_pml = static_cast<int>(pml_list.size());
    const int B = S.B;
    // slots of one class: consecutive, or with every component starting at a block boundary
    auto place = [&](const std::vector<int>& ord, int first_blk, std::vector<int>& c0, std::vector<int>& c1) {
        std::vector<int> slots(ord.size());
        int slot = first_blk * B;
        for (size_t i = 0; i < ord.size(); ++i) {
            if (align_components && i > 0 && comp[ord[i]] != comp[ord[i - 1]]) slot = (slot + B - 1) / B * B;
            slots[i] = slot++;
        }
        const int nblk_class = (slot - first_blk * B + B - 1) / B;
        if (align_components) {
            c0.assign(S.ncomp, 0);
            c1.assign(S.ncomp, 0);
            for (size_t i = 0; i < ord.size(); ++i) {
                const int c = comp[ord[i]], b = slots[i] / B;
                if (i == 0 || comp[ord[i - 1]] != c) c0[c] = b;
                c1[c] = b + 1;
            }
        }
        return std::make_pair(slots, nblk_class);
    };
    const auto pp = place(pml_order, 0, S.comp_pml0, S.comp_pml1);
    S.nblk_pml = pp.second;
    const auto ip = place(int_order, S.nblk_pml, S.comp_int0, S.comp_int1);
    S.nblk = S.nblk_pml + ip.second;
    S.perm.assign(K, -1);
    S.slot_elem.assign(static_cast<size_t>(S.nblk) * B, -1);
    for (size_t i = 0; i < pml_order.size(); ++i) {
        S.perm[pml_order[i]] = pp.first[i];
        S.slot_elem[pp.first[i]] = pml_order[i];
    }
    for (size_t i = 0; i < int_order.size(); ++i) {
        S.perm[int_order[i]] = ip.first[i];
        S.slot_elem[ip.first[i]] = int_order[i];
    }
    return S;
}

int locate_point(const Setup& S, const double* x, double* weights) {
    const RefElement& R = S.ref;
    int best = -1;
    double best_score = -1e300, br = 0, bs = 0, bt = 0;
    for (int k = 0; k < S.K; ++k) {
        const double* v0 = &S.vxyz[3 * static_cast<size_t>(S.etov[4 * static_cast<size_t>(k)])];
        const double* mt = &S.metric[9 * static_cast<size_t>(k)];
        double dx[3] = {x[0] - v0[0], x[1] - v0[1], x[2] - v0[2]};
        // (r+1, s+1, t+1) = grad(r,s,t) . (x - v0)
        const double rp = mt[0] * dx[0] + mt[1] * dx[1] + mt[2] * dx[2];
        const double sp = mt[3] * dx[0] + mt[4] * dx[1] + mt[5] * dx[2];
        const double tp = mt[6] * dx[0] + mt[7] * dx[1] + mt[8] * dx[2];
        const double l1 = 0.5 * rp, l2 = 0.5 * sp, l3 = 0.5 * tp, l0 = 1.0 - l1 - l2 - l3;
        const double score = std::min(std::min(l0, l1), std::min(l2, l3));
        if (score > best_score) {
            best_score = score;
            best = k;
            br = rp - 1.0;
            bs = sp - 1.0;
            bt = tp - 1.0;
        }
    }
    if (best < 0 || best_score < -1e-10) return -1;
    std::vector<double> phi(R.Np);
    ortho_basis(R.N, br, bs, bt, phi.data());
    // Lagrange weights l_j(x) = sum_m Vinv[m][j] phi_m(x)
    for (int j = 0; j < R.Np; ++j) {
        double acc = 0;
        for (int m = 0; m < R.Np; ++m) acc += R.Vinv[static_cast<size_t>(m) * R.Np + j] * phi[m];
        weights[j] = acc;
    }
    return best;
}

}  // namespace wdg
