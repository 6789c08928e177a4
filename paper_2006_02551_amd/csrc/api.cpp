// C ABI of the library (see include/wdg.h): context lifetime, device upload of
// the setup, state binding, stepping, readouts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/wdg.h"
#include "context.hpp"

using namespace wdg;

namespace {
thread_local std::string g_create_error;
}  // namespace

namespace wdg {

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Error(WDG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

std::vector<unsigned char> to_real(const std::vector<double>& v, int precision) {
    std::vector<unsigned char> out;
    if (precision == WDG_FP64) {
        out.resize(v.size() * sizeof(double));
        std::memcpy(out.data(), v.data(), out.size());
    } else {
        std::vector<float> f(v.begin(), v.end());
        out.resize(f.size() * sizeof(float));
        std::memcpy(out.data(), f.data(), out.size());
    }
    return out;
}

int fail(wdg_ctx* ctx, int code, const std::string& msg) {
    if (ctx)
        ctx->err = msg;
    else
        g_create_error = msg;
    return code;
}

int64_t state_index(const Setup& S, int k, int c, int i) {
    const int slot = S.perm[k];
    const int blk = slot / S.B, lane = slot % S.B;
    const int64_t ehs = eh_words(S);
    if (c < 6) return blk * ehs + (static_cast<int64_t>(c) * S.ref.Np + i) * S.B + lane;
    if (!S.is_pml[k]) return -1;
    return static_cast<int64_t>(S.nblk) * ehs + blk * ehs + (static_cast<int64_t>(c - 6) * S.ref.Np + i) * S.B + lane;
}

}  // namespace wdg

namespace wdg {

void upload_coefficients(wdg_ctx* c) {
    const Setup& S = c->S;
    const int Nq = S.ref.Nq, B = S.B, nblk_pml = S.nblk_pml;
    // sigma (and kappa) at cubature points, PML blocks only
    std::vector<double> sg(static_cast<size_t>(std::max(nblk_pml, 1)) * 3 * Nq * B, 0.0);
    std::vector<double> kp(S.has_kappa ? sg.size() : 0, 1.0);
    for (int slot = 0; slot < nblk_pml * B; ++slot) {
        const int k = S.slot_elem[slot];
        if (k < 0) continue;
        const int blk = slot / B, lane = slot % B;
        for (int d = 0; d < 3; ++d)
            for (int q = 0; q < Nq; ++q) {
                const size_t di = ((static_cast<size_t>(blk) * 3 + d) * Nq + q) * B + lane;
                sg[di] = S.sigma[(static_cast<size_t>(k) * Nq + q) * 3 + d];
                if (S.has_kappa) kp[di] = S.kappa[(static_cast<size_t>(k) * Nq + q) * 3 + d];
            }
    }
    c->drop_graph();
    c->sigma.upload(to_real(sg, c->precision).data(), sg.size() * c->rsize);
    if (S.has_kappa) c->kappa.upload(to_real(kp, c->precision).data(), kp.size() * c->rsize);
}

}  // namespace wdg

namespace {

void upload_setup(wdg_ctx* c) {
    const Setup& S = c->S;
    const RefElement& R = S.ref;
    const int Np = R.Np, Nfp = R.Nfp, Nq = R.Nq, B = S.B, nblk = S.nblk, nblk_pml = S.nblk_pml;
    const int64_t ehs = eh_words(S);
    // geometry
    std::vector<double> geo(static_cast<size_t>(nblk) * kGeo * B, 0.0);
    std::vector<int> nbr(static_cast<size_t>(nblk) * 4 * Nfp * B, 0);
    std::vector<double> Jk(static_cast<size_t>(nblk) * B, 0.0);
    for (int slot = 0; slot < nblk * B; ++slot) {
        const int blk = slot / B, lane = slot % B;
        const int k = S.slot_elem[slot];
        const int64_t own_base = blk * ehs + lane;
        for (int f = 0; f < 4; ++f)
            for (int m = 0; m < Nfp; ++m) {
                const size_t ni = (static_cast<size_t>(blk) * 4 * Nfp + f * Nfp + m) * B + lane;
                const int jn = R.fmask[f * Nfp + m];
                if (k < 0) {  // padding slot: a wall onto itself, zero geometry
                    nbr[ni] = ~static_cast<int>(own_base + static_cast<int64_t>(jn) * B);
                    continue;
                }
                const int k2 = S.etoe[4 * static_cast<size_t>(k) + f];
                const int j2 = S.nbr_node[(static_cast<size_t>(k) * 4 + f) * Nfp + m];
                if (k2 == k) {
                    nbr[ni] = ~static_cast<int>(own_base + static_cast<int64_t>(jn) * B);
                } else {
                    const int s2 = S.perm[k2];
                    nbr[ni] = static_cast<int>((s2 / B) * ehs + static_cast<int64_t>(j2) * B + (s2 % B));
                }
            }
        if (k < 0) continue;
        for (int d = 0; d < 9; ++d) geo[(static_cast<size_t>(blk) * kGeo + d) * B + lane] = S.metric[9 * static_cast<size_t>(k) + d];
        for (int f = 0; f < 4; ++f) {
            for (int d = 0; d < 3; ++d)
                geo[(static_cast<size_t>(blk) * kGeo + 9 + 4 * f + d) * B + lane] = S.nrm[12 * static_cast<size_t>(k) + 3 * f + d];
            geo[(static_cast<size_t>(blk) * kGeo + 12 + 4 * f) * B + lane] = S.Fscale[4 * static_cast<size_t>(k) + f];
        }
        Jk[slot] = S.J[k];
    }
    c->geo.upload(to_real(geo, c->precision).data(), geo.size() * c->rsize);
    c->nbr.upload(nbr.data(), nbr.size() * sizeof(int));
    c->Jk.upload(Jk.data(), Jk.size() * sizeof(double));

    upload_coefficients(c);

    // operators packed in one buffer
    std::vector<double> ops;
    auto push = [&](const Mat& m) {
        const size_t off = ops.size();
        ops.insert(ops.end(), m.begin(), m.end());
        return off;
    };
    c->off_DrT = push(transpose(R.Dr, Np, Np));
    c->off_DsT = push(transpose(R.Ds, Np, Np));
    c->off_DtT = push(transpose(R.Dt, Np, Np));
    c->off_LIFTT = push(transpose(R.LIFT, Np, 4 * Nfp));
    c->off_Vq = push(R.Vq);
    c->off_PqT = push(transpose(R.Pq, Np, Nq));
    c->ops.upload(to_real(ops, c->precision).data(), ops.size() * c->rsize);

    // With kappa = 1 the coefficient a of eq. (9) is one, and P_q a^-1 V_q = P_q V_q = M^-1 V_q^T W V_q
    // is the identity whenever the rule integrates products of two degree-N polynomials exactly.
    {
        const Mat PV = matmul(R.Pq, R.Vq, Np, Nq, Np);
        double dev = 0.0;
        for (int i = 0; i < Np; ++i)
            for (int jj = 0; jj < Np; ++jj) dev = std::max(dev, std::fabs(PV[i * Np + jj] - (i == jj ? 1.0 : 0.0)));
        c->waa_identity = !S.has_kappa && dev < 1e-12;
    }

    // MFMA A-operand fragments (layout in device.hpp): V_q with full tiles (its
    // row count N_q is a run-time value in the kernel), then P_q, D_r, D_s, D_t
    // and LIFT, whose last tile of N_p rows is stored compact.
    // (the matrix-core kernel addresses neighbour traces with 32-bit byte offsets into the E,H part)
    c->mfma_ok = mfma_supported(R.N, Nq, c->precision) &&
                 static_cast<double>(S.nblk) * eh_words(S) * c->rsize < 4294967296.0;
    // two tiles per workgroup where they fit in LDS (FP64 at N = 4 takes one)
    if (c->mfma_ok && !mfma_tiles_fit(R.N, Nq, c->precision, c->tpw)) c->tpw = 1;
    if (c->mfma_ok) {
        const int PT = (Np + 15) / 16, SP = (Np + 3) / 4, QT = (Nq + 15) / 16, SQM = 4 * QT, SF = Nfp;
        const bool f64 = c->precision == WDG_FP64;
        auto qloc = [&](int rr) { return f64 ? rr : 4 * (rr % 4) + rr / 4; };
        std::vector<double> fr;
        auto add = [&](const Mat& X, int rows, int cols, int tiles, int ksteps, bool compact) {
            const size_t start = fr.size();
            auto val = [&](int row, int col) { return row < rows && col < cols ? X[static_cast<size_t>(row) * cols + col] : 0.0; };
            for (int t = 0; t < tiles; ++t)
                for (int ks = 0; ks < ksteps; ++ks) {
                    if (f64) {
                        // four-block 4x4x4 products: word (k, i, v) holds row 16 t + 4 v + i, column 4 ks + k
                        const int nv = (compact && t == tiles - 1) ? (rows - 16 * t + 3) / 4 : 4;
                        for (int k = 0; k < 4; ++k)
                            for (int i = 0; i < 4; ++i)
                                for (int v = 0; v < nv; ++v) fr.push_back(val(16 * t + 4 * v + i, 4 * ks + k));
                    } else if (compact && t == tiles - 1) {
                        const int m = rows - 16 * t;
                        for (int k = 0; k < 4; ++k)
                            for (int i = 0; i < m; ++i) {
                                const int col = 4 * ks + k;
                                fr.push_back(col < cols ? X[static_cast<size_t>(16 * t + i) * cols + col] : 0.0);
                            }
                    } else {
                        for (int l = 0; l < 64; ++l) {
                            const int row = 16 * t + qloc(l % 16), col = 4 * ks + l / 16;
                            fr.push_back(row < rows && col < cols ? X[static_cast<size_t>(row) * cols + col] : 0.0);
                        }
                    }
                }
            if (fr.size() - start != static_cast<size_t>(frag_words(rows, tiles, ksteps, compact, f64)))
                throw std::logic_error("fragment size");
        };
        add(R.Vq, Nq, Np, QT, SP, false);
        add(R.Pq, Np, Nq, PT, SQM, true);
        add(R.Dr, Np, Np, PT, SP, true);
        add(R.Ds, Np, Np, PT, SP, true);
        add(R.Dt, Np, Np, PT, SP, true);
        add(R.LIFT, Np, 4 * Nfp, PT, SF, true);
        // padded to whole 1 KiB chunks (the kernel copies it with 16-byte direct loads into LDS)
        fr.resize(static_cast<size_t>(frag_chunks(static_cast<int>(fr.size()), static_cast<int>(c->rsize))) * 1024 / c->rsize, 0.0);
        c->frags.upload(to_real(fr, c->precision).data(), fr.size() * c->rsize);
        c->kernel = WDG_KERNEL_MFMA;
    }
    // environment overrides of the stage-kernel choice (checked like wdg_set_kernel / wdg_set_tiles)
    if (const char* k = std::getenv("WDG_KERNEL")) {
        if (std::strcmp(k, "scalar") == 0)
            c->kernel = WDG_KERNEL_SCALAR;
        else if (std::strcmp(k, "mfma") == 0 && c->mfma_ok)
            c->kernel = WDG_KERNEL_MFMA;
        else
            throw Error(WDG_EINVAL, std::string("WDG_KERNEL=") + k + ": expected scalar, or mfma where available");
    }
    if (const char* t = std::getenv("WDG_TILES")) {
        const int tiles = std::strcmp(t, "1") == 0 ? 1 : std::strcmp(t, "2") == 0 ? 2 : 0;
        if (tiles == 0 || (c->mfma_ok && !mfma_tiles_fit(R.N, Nq, c->precision, tiles)))
            throw Error(WDG_EINVAL, std::string("WDG_TILES=") + t + ": expected 1 or 2 tiles that fit in a compute unit");
        c->tpw = tiles;
    }
    c->fmask.upload(R.fmask.data(), R.fmask.size() * sizeof(int));
    c->cubw.upload(R.wq.data(), R.wq.size() * sizeof(double));
    c->Mref.upload(R.M.data(), R.M.size() * sizeof(double));
    c->partial.alloc(static_cast<size_t>(nblk) * sizeof(double));
    c->scalar_out.alloc(sizeof(double));
    std::vector<int> slots(nblk, -1);
    c->src_slot.upload(slots.data(), slots.size() * sizeof(int));
}

}  // namespace

namespace wdg {

int launch_stage_on(wdg_ctx* c, const void* qin, void* qout, void* res, double rk_a, double rk_b, double dt, double t,
                    bool read_res, hipStream_t stream) {
    const Setup& S = c->S;
    StageParams p{};
    p.q_in = qin;
    p.q_out = qout;
    p.res = res;
    p.geo = c->geo.p;
    p.nbr = static_cast<const int*>(c->nbr.p);
    p.sigma = c->sigma.p;
    p.kappa = c->kappa.p;
    p.DrT = cptr(c->ops, c->off_DrT, c->rsize);
    p.DsT = cptr(c->ops, c->off_DsT, c->rsize);
    p.DtT = cptr(c->ops, c->off_DtT, c->rsize);
    p.LIFTT = cptr(c->ops, c->off_LIFTT, c->rsize);
    p.Vq = cptr(c->ops, c->off_Vq, c->rsize);
    p.PqT = cptr(c->ops, c->off_PqT, c->rsize);
    p.fmask = static_cast<const int*>(c->fmask.p);
    p.src_slot = static_cast<const int*>(c->src_slot.p);
    p.src = c->src.p;
    p.frags = c->frags.p;
    p.dt_scale = c->has_dt_scale ? static_cast<const double*>(c->dt_scale.p) : nullptr;
    p.pml_mats = c->pml_mats.p;
    p.pml_work = c->pml_work.p;
    p.waa_skip = (c->waa_skip && c->waa_identity) ? 1 : 0;
    p.nblk_pml = S.nblk_pml;
    p.nblk = S.nblk;
    if (c->range_on) {  // one group of independent simulations (captured grouped stepping)
        p.pml0 = c->range[0];
        p.npml = c->range[1];
        p.int0 = c->range[2];
        p.nint = c->range[3];
    } else {
        p.pml0 = 0;
        p.npml = S.nblk_pml;
        p.int0 = S.nblk_pml;
        p.nint = S.nblk - S.nblk_pml;
    }
    p.Nq = S.ref.Nq;
    p.read_res = read_res ? 1 : 0;
    p.order_rev = c->next_order_rev();
    p.rk_a = rk_a;
    p.rk_b = rk_b;
    p.dt = dt;
    p.alpha = S.flux_alpha;
    p.src_g = 0.0;
    if (c->has_src) {
        const wdg_dipole& d = c->dip;
        const double tt = t - d.t0;
        p.src_g = d.amplitude * std::sin(2.0 * M_PI * d.f0 * tt) * std::exp(-(tt / d.tau) * (tt / d.tau));
    }
    const int e = c->kernel == WDG_KERNEL_MFMA ? launch_stage_mfma(c->precision, S.ref.N, S.has_kappa, c->tpw, c->pml_scheme, p, stream)
                                               : launch_stage(c->precision, S.ref.N, S.has_kappa, c->pml_scheme, p, stream);
    if (e != 0) return fail(c, WDG_EHIP, std::string("stage launch: ") + hipGetErrorString(static_cast<hipError_t>(e)));
    return WDG_OK;
}

int check_state(wdg_ctx* c) {
    if (c->host_only) return fail(c, WDG_ESTATE, "host-only context");
    if (!c->q[0] || !c->q[1] || !c->res) return fail(c, WDG_ESTATE, "state buffers not bound");
    return WDG_OK;
}

}  // namespace wdg

extern "C" {

int32_t wdg_version(void) { return 10000; }

const char* wdg_error_string(int32_t code) {
    switch (code) {
        case WDG_OK: return "ok";
        case WDG_EINVAL: return "invalid argument";
        case WDG_EMESH: return "invalid mesh";
        case WDG_ENOMEM: return "out of memory";
        case WDG_EHIP: return "HIP runtime error";
        case WDG_ESTATE: return "state not bound or host-only context";
        case WDG_EPROBE: return "probe error";
        case WDG_ENONFINITE: return "non-finite energy";
        default: return "unknown error";
    }
}

const char* wdg_last_error(const wdg_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int32_t wdg_create(const wdg_mesh* mesh, const wdg_method* m, wdg_ctx** out) {
    if (!out) return fail(nullptr, WDG_EINVAL, "null output pointer");
    *out = nullptr;
    if (!mesh || !m) return fail(nullptr, WDG_EINVAL, "null mesh or method");
    if (m->precision != WDG_FP64 && m->precision != WDG_FP32) return fail(nullptr, WDG_EINVAL, "precision");
    if (m->nq < 1 || m->nq > 128) return fail(nullptr, WDG_EINVAL, "nq must be 1..128");
    if (mesh->K <= 0 || mesh->nv <= 0) return fail(nullptr, WDG_EMESH, "empty mesh");
    for (int d = 0; d < 3; ++d)
        if (!(m->pml_L[d] > 0.0) || m->sigma_max[d] < 0.0 || m->pml_hi[d] < m->pml_lo[d])
            return fail(nullptr, WDG_EINVAL, "PML parameters");
    if (!(m->kappa_max >= 1.0) || m->profile_order < 0.0) return fail(nullptr, WDG_EINVAL, "PML profile");
    auto ctx = std::make_unique<wdg_ctx>();
    const int rc = guarded(nullptr, [&]() -> int {
        PmlParams pp{};
        for (int d = 0; d < 3; ++d) {
            pp.lo[d] = m->pml_lo[d];
            pp.hi[d] = m->pml_hi[d];
            pp.L[d] = m->pml_L[d];
            pp.sigma_max[d] = m->sigma_max[d];
        }
        pp.order = m->profile_order;
        pp.kappa_max = m->kappa_max;
        ctx->S = build_setup(mesh->nv, mesh->vxyz, mesh->K, mesh->etov, mesh->vertex_id, m->N, m->nq, m->cub_rst,
                             m->cub_w, pp, m->flux_alpha, (m->flags & WDG_ALIGN_COMPONENTS) != 0);
        // neighbour traces are addressed by 32-bit signed word offsets into the E,H part
        if (static_cast<int64_t>(ctx->S.nblk) * eh_words(ctx->S) > kMaxEhWords)
            throw Error(WDG_EINVAL, "mesh too large: the E,H part exceeds 2^31 - 1 words (32-bit neighbour offsets)");
        ctx->precision = m->precision;
        ctx->rsize = m->precision == WDG_FP64 ? sizeof(double) : sizeof(float);
        ctx->host_only = (m->flags & WDG_HOST_ONLY) != 0;
        ctx->state_elems = (static_cast<int64_t>(ctx->S.nblk) + ctx->S.nblk_pml) * eh_words(ctx->S);
        if (!ctx->host_only) {
            hip_check(hipGetDevice(&ctx->device), "hipGetDevice");
            hip_check(static_cast<hipError_t>(noalloc_setup(ctx->device)), "scratch symbol address");
            upload_setup(ctx.get());
        }
        return WDG_OK;
    });
    if (rc != WDG_OK) return rc;
    *out = ctx.release();
    return WDG_OK;
}

void wdg_destroy(wdg_ctx* ctx) { delete ctx; }

int32_t wdg_get_dims(const wdg_ctx* c, wdg_dims_t* o) {
    if (!c || !o) return WDG_EINVAL;
    const Setup& S = c->S;
    o->K = S.K;
    o->K_pml = S.K_pml;
    o->N = S.ref.N;
    o->Np = S.ref.Np;
    o->Nfp = S.ref.Nfp;
    o->Nq = S.ref.Nq;
    o->block = S.B;
    o->nblk_pml = S.nblk_pml;
    o->nblk = S.nblk;
    o->precision = c->precision;
    o->has_kappa = S.has_kappa ? 1 : 0;
    o->state_bytes = c->state_elems * static_cast<int64_t>(c->rsize);
    o->dt_unit = S.dt_unit;
    o->time = c->t;
    o->steps = c->steps;
    o->kernel = c->kernel;
    o->tiles = c->tpw;
    o->pml_scheme = c->pml_scheme;
    return WDG_OK;
}

int32_t wdg_set_kernel(wdg_ctx* c, int32_t variant) {
    if (!c) return WDG_EINVAL;
    if (c->host_only) return fail(c, WDG_ESTATE, "host-only context");
    if (variant == WDG_KERNEL_AUTO) variant = c->mfma_ok ? WDG_KERNEL_MFMA : WDG_KERNEL_SCALAR;
    if (variant == WDG_KERNEL_MFMA && !c->mfma_ok) return fail(c, WDG_EINVAL, "no MFMA kernel for this order and rule size");
    if (variant != WDG_KERNEL_MFMA && variant != WDG_KERNEL_SCALAR) return fail(c, WDG_EINVAL, "unknown kernel variant");
    c->kernel = variant;
    return WDG_OK;
}

int32_t wdg_bind_state(wdg_ctx* c, void* q0, void* q1, void* res, int64_t bytes_each) {
    if (!c) return WDG_EINVAL;
    if (c->host_only) return fail(c, WDG_ESTATE, "host-only context");
    if (!q0 || !q1 || !res) return fail(c, WDG_EINVAL, "null state buffer");
    for (const void* b : {static_cast<const void*>(q0), static_cast<const void*>(q1), static_cast<const void*>(res)})
        if (reinterpret_cast<uintptr_t>(b) % 16 != 0) return fail(c, WDG_EINVAL, "state buffer not 16-byte aligned");
    if (bytes_each < c->state_elems * static_cast<int64_t>(c->rsize)) return fail(c, WDG_EINVAL, "state buffers too small");
    c->q[0] = q0;
    c->q[1] = q1;
    c->res = res;
    c->cur = 0;
    return WDG_OK;
}

int32_t wdg_set_fields(wdg_ctx* c, const double* q) {
    if (!c || !q) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    return guarded(c, [&]() -> int {
        const Setup& S = c->S;
        const int Np = S.ref.Np;
        std::vector<double> buf(static_cast<size_t>(c->state_elems), 0.0);
        for (int k = 0; k < S.K; ++k)
            for (int comp = 0; comp < 12; ++comp)
                for (int i = 0; i < Np; ++i) {
                    const int64_t idx = state_index(S, k, comp, i);
                    if (idx >= 0) buf[idx] = q[(static_cast<size_t>(k) * 12 + comp) * Np + i];
                }
        const auto bytes = to_real(buf, c->precision);
        hip_check(hipDeviceSynchronize(), "sync");
        hip_check(hipMemcpy(c->q[c->cur], bytes.data(), bytes.size(), hipMemcpyHostToDevice), "upload fields");
        hip_check(hipMemset(c->res, 0, bytes.size()), "clear residual");
        hip_check(hipMemset(c->q[1 - c->cur], 0, bytes.size()), "clear second buffer");
        c->steps = 0;
        c->probe_rows = 0;
        return WDG_OK;
    });
}

static int download(wdg_ctx* c, const void* dev, double* q) {
    const Setup& S = c->S;
    const int Np = S.ref.Np;
    hip_check(hipDeviceSynchronize(), "sync");
    std::vector<unsigned char> raw(static_cast<size_t>(c->state_elems) * c->rsize);
    hip_check(hipMemcpy(raw.data(), dev, raw.size(), hipMemcpyDeviceToHost), "download fields");
    for (int k = 0; k < S.K; ++k)
        for (int comp = 0; comp < 12; ++comp)
            for (int i = 0; i < Np; ++i) {
                const int64_t idx = state_index(S, k, comp, i);
                double v = 0.0;
                if (idx >= 0)
                    v = c->precision == WDG_FP64 ? reinterpret_cast<const double*>(raw.data())[idx]
                                                 : static_cast<double>(reinterpret_cast<const float*>(raw.data())[idx]);
                q[(static_cast<size_t>(k) * 12 + comp) * Np + i] = v;
            }
    return WDG_OK;
}

int32_t wdg_get_fields(wdg_ctx* c, double* q) {
    if (!c || !q) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    return guarded(c, [&]() -> int { return download(c, c->q[c->cur], q); });
}

int32_t wdg_get_residual(wdg_ctx* c, double* r) {
    if (!c || !r) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    return guarded(c, [&]() -> int { return download(c, c->res, r); });
}

int32_t wdg_set_time(wdg_ctx* c, double t) {
    if (!c) return WDG_EINVAL;
    c->t = t;
    return WDG_OK;
}

int32_t wdg_set_dipole(wdg_ctx* c, const wdg_dipole* d) {
    if (!c) return WDG_EINVAL;
    if (c->host_only) return fail(c, WDG_ESTATE, "host-only context");
    return guarded(c, [&]() -> int {
        const Setup& S = c->S;
        const int Np = S.ref.Np, B = S.B;
        std::vector<int> slots(S.nblk, -1);
        c->has_src = false;
        if (!d) {
            hip_check(hipMemcpy(c->src_slot.p, slots.data(), slots.size() * sizeof(int), hipMemcpyHostToDevice), "src");
            return WDG_OK;
        }
        if (!(d->width > 0.0) || !(d->tau > 0.0)) return fail(c, WDG_EINVAL, "dipole width and tau must be positive");
        // spatial factor at the nodes; keep elements where it reaches 1e-16 somewhere
        std::vector<char> use(S.K, 0);
        for (int k = 0; k < S.K; ++k)
            for (int i = 0; i < Np; ++i) {
                const double* x = &S.xnodes[(static_cast<size_t>(k) * Np + i) * 3];
                double r2 = 0;
                for (int dd = 0; dd < 3; ++dd) r2 += (x[dd] - d->center[dd]) * (x[dd] - d->center[dd]);
                if (std::exp(-r2 / (d->width * d->width)) >= 1e-16) use[k] = 1;
            }
        int nslot = 0;
        for (int blk = 0; blk < S.nblk; ++blk)
            for (int lane = 0; lane < B; ++lane) {
                const int k = S.slot_elem[static_cast<size_t>(blk) * B + lane];
                if (k >= 0 && use[k]) {
                    slots[blk] = nslot++;
                    break;
                }
            }
        std::vector<double> src(static_cast<size_t>(std::max(nslot, 1)) * 3 * Np * B, 0.0);
        for (int blk = 0; blk < S.nblk; ++blk) {
            if (slots[blk] < 0) continue;
            for (int lane = 0; lane < B; ++lane) {
                const int k = S.slot_elem[static_cast<size_t>(blk) * B + lane];
                if (k < 0 || !use[k]) continue;
                for (int i = 0; i < Np; ++i) {
                    const double* x = &S.xnodes[(static_cast<size_t>(k) * Np + i) * 3];
                    double r2 = 0;
                    for (int dd = 0; dd < 3; ++dd) r2 += (x[dd] - d->center[dd]) * (x[dd] - d->center[dd]);
                    const double sp = std::exp(-r2 / (d->width * d->width));
                    for (int comp = 0; comp < 3; ++comp)
                        src[((static_cast<size_t>(slots[blk]) * 3 + comp) * Np + i) * B + lane] = sp * d->direction[comp];
                }
            }
        }
        c->drop_graph();
        c->src.upload(to_real(src, c->precision).data(), src.size() * c->rsize);
        hip_check(hipMemcpy(c->src_slot.p, slots.data(), slots.size() * sizeof(int), hipMemcpyHostToDevice), "src");
        c->dip = *d;
        c->has_src = true;
        return WDG_OK;
    });
}

int32_t wdg_set_probes(wdg_ctx* c, int32_t n, const double* xyz, int32_t capacity) {
    if (!c || n < 0 || (n > 0 && (!xyz || capacity <= 0)) || n > 160) return WDG_EINVAL;
    if (c->host_only) return fail(c, WDG_ESTATE, "host-only context");
    return guarded(c, [&]() -> int {
        const Setup& S = c->S;
        const int Np = S.ref.Np;
        c->nprobe = 0;
        c->probe_rows = 0;
        if (n == 0) return WDG_OK;
        std::vector<int> slot(n);
        std::vector<double> w(static_cast<size_t>(n) * Np);
        for (int p = 0; p < n; ++p) {
            const int k = locate_point(S, xyz + 3 * p, &w[static_cast<size_t>(p) * Np]);
            if (k < 0) return fail(c, WDG_EPROBE, "probe point outside the mesh");
            slot[p] = S.perm[k];
        }
        c->probe_slot.upload(slot.data(), slot.size() * sizeof(int));
        c->probe_w.upload(w.data(), w.size() * sizeof(double));
        c->probe_buf.alloc(static_cast<size_t>(capacity) * n * 6 * sizeof(double));
        c->nprobe = n;
        c->probe_cap = capacity;
        return WDG_OK;
    });
}

int32_t wdg_probe_read(wdg_ctx* c, double* out, int32_t max_rows, int32_t* nrows) {
    if (!c || !nrows) return WDG_EINVAL;
    if (c->host_only) return fail(c, WDG_ESTATE, "host-only context");
    return guarded(c, [&]() -> int {
        const int rows = std::min(c->probe_rows, std::max(max_rows, 0));
        *nrows = rows;
        if (rows > 0) {
            if (!out) return fail(c, WDG_EINVAL, "null output");
            hip_check(hipDeviceSynchronize(), "sync");
            hip_check(hipMemcpy(out, c->probe_buf.p, static_cast<size_t>(rows) * c->nprobe * 6 * sizeof(double),
                                hipMemcpyDeviceToHost),
                      "probe download");
        }
        c->probe_rows = 0;
        return WDG_OK;
    });
}

int32_t wdg_step(wdg_ctx* c, double dt, int32_t nsteps, void* hip_stream) {
    if (!c || nsteps < 0 || !(std::isfinite(dt))) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    if (c->nprobe > 0 && c->probe_rows + nsteps > c->probe_cap) return fail(c, WDG_EPROBE, "probe buffer would overflow");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    TraceRange range("wdg_step");
    return guarded(c, [&]() -> int {
        for (int n = 0; n < nsteps; ++n) {
            TraceRange step("step");
            for (int i = 0; i < 5; ++i) {
                const int rc = launch_stage_on(c, c->q[c->cur], c->q[1 - c->cur], c->res, kRkA[i], kRkB[i], dt,
                                               c->t + kRkC[i] * dt, i > 0, s);
                if (rc != WDG_OK) return rc;
                c->cur = 1 - c->cur;
            }
            c->t += dt;
            c->steps += 1;
            if (c->nprobe > 0) {
                ProbeParams pp{};
                pp.q = c->q[c->cur];
                pp.slot = static_cast<const int*>(c->probe_slot.p);
                pp.w = static_cast<const double*>(c->probe_w.p);
                pp.out = static_cast<double*>(c->probe_buf.p) + static_cast<size_t>(c->probe_rows) * c->nprobe * 6;
                pp.n = c->nprobe;
                const int e = launch_probe(c->precision, c->S.ref.N, pp, s);
                if (e != 0) return fail(c, WDG_EHIP, "probe launch");
                c->probe_rows += 1;
            }
        }
        return WDG_OK;
    });
}

int32_t wdg_rhs(wdg_ctx* c, double t, void* hip_stream) {
    if (!c) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return guarded(c, [&]() -> int {
        // res = 0 * res + 1 * rhs, q_out = q_in + 0 * res into the spare buffer
        return launch_stage_on(c, c->q[c->cur], c->q[1 - c->cur], c->res, 0.0, 0.0, 1.0, t, false, s);
    });
}

int32_t wdg_energy(wdg_ctx* c, double* out, void* hip_stream) {
    if (!c || !out) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return guarded(c, [&]() -> int {
        EnergyParams p{};
        p.q = c->q[c->cur];
        p.J = static_cast<const double*>(c->Jk.p);
        p.M = static_cast<const double*>(c->Mref.p);
        p.partial = static_cast<double*>(c->partial.p);
        p.nblk = c->S.nblk;
        const int e = launch_energy(c->precision, c->S.ref.N, p, static_cast<double*>(c->scalar_out.p), s);
        if (e != 0) return fail(c, WDG_EHIP, "energy launch");
        hip_check(hipMemcpyAsync(out, c->scalar_out.p, sizeof(double), hipMemcpyDeviceToHost, s), "energy download");
        hip_check(hipStreamSynchronize(s), "energy sync");
        if (!std::isfinite(*out)) return fail(c, WDG_ENONFINITE, "energy is not finite");
        return WDG_OK;
    });
}

int32_t wdg_element_slots(const wdg_ctx* c, int32_t* slot) {
    if (!c || !slot) return WDG_EINVAL;
    std::copy(c->S.perm.begin(), c->S.perm.end(), slot);
    return WDG_OK;
}

int32_t wdg_node_coords(const wdg_ctx* c, double* xyz) {
    if (!c || !xyz) return WDG_EINVAL;
    std::memcpy(xyz, c->S.xnodes.data(), c->S.xnodes.size() * sizeof(double));
    return WDG_OK;
}

int32_t wdg_reference_op(const wdg_ctx* c, int32_t which, double* out) {
    if (!c || !out) return WDG_EINVAL;
    const RefElement& R = c->S.ref;
    const Mat* m = nullptr;
    switch (which) {
        case WDG_OP_DR: m = &R.Dr; break;
        case WDG_OP_DS: m = &R.Ds; break;
        case WDG_OP_DT: m = &R.Dt; break;
        case WDG_OP_LIFT: m = &R.LIFT; break;
        case WDG_OP_VQ: m = &R.Vq; break;
        case WDG_OP_PQ: m = &R.Pq; break;
        case WDG_OP_M: m = &R.M; break;
        default: return WDG_EINVAL;
    }
    std::memcpy(out, m->data(), m->size() * sizeof(double));
    return WDG_OK;
}

int32_t wdg_element_info(const wdg_ctx* c, double* J, double* Fscale, double* normals, int32_t* etoe, int32_t* etof,
                         int32_t* is_pml) {
    if (!c) return WDG_EINVAL;
    const Setup& S = c->S;
    if (J) std::memcpy(J, S.J.data(), S.J.size() * sizeof(double));
    if (Fscale) std::memcpy(Fscale, S.Fscale.data(), S.Fscale.size() * sizeof(double));
    if (normals) std::memcpy(normals, S.nrm.data(), S.nrm.size() * sizeof(double));
    if (etoe) std::memcpy(etoe, S.etoe.data(), S.etoe.size() * sizeof(int));
    if (etof) std::memcpy(etof, S.etof.data(), S.etof.size() * sizeof(int));
    if (is_pml) std::memcpy(is_pml, S.is_pml.data(), S.is_pml.size() * sizeof(int));
    return WDG_OK;
}

int32_t wdg_memory_report(const wdg_ctx* c, wdg_mem_t* o) {
    if (!c || !o) return WDG_EINVAL;
    const Setup& S = c->S;
    const int64_t r = static_cast<int64_t>(c->rsize);
    const int64_t Np = S.ref.Np, Nq = S.ref.Nq, B = S.B;
    o->state = 3 * c->state_elems * r;
    o->geometry = static_cast<int64_t>(S.nblk) * B * (kGeo * r + static_cast<int64_t>(sizeof(double)));
    o->connectivity = static_cast<int64_t>(S.nblk) * B * 4 * S.ref.Nfp * static_cast<int64_t>(sizeof(int));
    o->coefficients = static_cast<int64_t>(S.nblk_pml) * B * 3 * Nq * r * (S.has_kappa ? 2 : 1);
    o->operators = (3 * Np * Np + Np * 4 * S.ref.Nfp + 2 * Np * Nq) * r;
    o->paper_direct = 15 * Np * Np * static_cast<int64_t>(S.K_pml) * 8;
    o->paper_waa = (15 * Nq * static_cast<int64_t>(S.K_pml) + 2 * Np * Nq) * 8;
    o->scheme_data = static_cast<int64_t>(c->pml_mats.bytes + c->pml_work.bytes);
    return WDG_OK;
}

}  // extern "C"
