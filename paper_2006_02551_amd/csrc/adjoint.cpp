// Differentiation through the time-stepped scheme (C ABI part): the sigma
// override and readouts, the shell-energy loss, and the loss gradient by the
// discrete adjoint of the LSERK4 / weight-adjusted SC-PML scheme.
//
// The adjoint runs in the energy inner product <x, y> = sum_k J_k x^T M y, in
// which the adjoint of a stage is the adjoint stage kernel (the vacuum
// operator with the flux parameter negated, the PML terms transposed) applied
// to z = P_q a^{-1} V_q y.  The stages of a step are reversed as
//     y <- A_{i+1} y + B_i q_hat   (A_6 = 0),   q_hat <- q_hat + dt L* y,
// each needing the forward stage input for the sigma gradient.  Forward
// states are checkpointed every C steps (C = ceil(sqrt(nsteps)) by default);
// each segment is recomputed from its checkpoint keeping all 5 C + 1 stage
// inputs, then reversed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "context.hpp"

using namespace wdg;

namespace {

// Blocks that hold shell cubature points and the shell indicator there.
struct ShellDev {
    DevBuf blocks, chi, partial;
    int nsb = 0;
};

bool in_shell(const wdg_shell& sh, const double* x) {
    bool in_outer = true, in_inner = true;
    for (int d = 0; d < 3; ++d) {
        in_outer = in_outer && x[d] >= sh.outer_lo[d] && x[d] <= sh.outer_hi[d];
        in_inner = in_inner && x[d] > sh.inner_lo[d] && x[d] < sh.inner_hi[d];
    }
    return in_outer && !in_inner;
}

void build_shell(wdg_ctx* c, const wdg_shell& sh, ShellDev& out) {
    const Setup& S = c->S;
    const int Nq = S.ref.Nq, B = S.B;
    std::vector<int> blocks;
    std::vector<double> chi;
    std::vector<double> cb(static_cast<size_t>(Nq) * B);
    for (int blk = 0; blk < S.nblk; ++blk) {
        std::fill(cb.begin(), cb.end(), 0.0);
        bool any = false;
        for (int lane = 0; lane < B; ++lane) {
            const int k = S.slot_elem[static_cast<size_t>(blk) * B + lane];
            if (k < 0) continue;
            for (int q = 0; q < Nq; ++q)
                if (in_shell(sh, &S.xq[(static_cast<size_t>(k) * Nq + q) * 3])) {
                    cb[static_cast<size_t>(q) * B + lane] = 1.0;
                    any = true;
                }
        }
        if (any) {
            blocks.push_back(blk);
            chi.insert(chi.end(), cb.begin(), cb.end());
        }
    }
    out.nsb = static_cast<int>(blocks.size());
    out.blocks.upload(blocks.data(), blocks.size() * sizeof(int));
    out.chi.upload(to_real(chi, c->precision).data(), chi.size() * c->rsize);
    out.partial.alloc(static_cast<size_t>(std::max(out.nsb, 1)) * sizeof(double));
}

ShellParams shell_params(wdg_ctx* c, const ShellDev& sd, const void* q, void* qhat, double dt) {
    ShellParams p{};
    p.q = q;
    p.q_hat = qhat;
    p.blocks = static_cast<const int*>(sd.blocks.p);
    p.chi = sd.chi.p;
    p.Jk = static_cast<const double*>(c->Jk.p);
    p.cub_w = static_cast<const double*>(c->cubw.p);
    p.Vq = cptr(c->ops, c->off_Vq, c->rsize);
    p.PqT = cptr(c->ops, c->off_PqT, c->rsize);
    p.partial = static_cast<double*>(sd.partial.p);
    p.nsb = sd.nsb;
    p.nblk = c->S.nblk;
    p.Nq = c->S.ref.Nq;
    p.dt = dt;
    return p;
}

// acc += scale * shell_energy(q)
void shell_energy_into(wdg_ctx* c, const ShellDev& sd, const void* q, double scale, double* acc, hipStream_t s) {
    if (sd.nsb == 0) return;
    const ShellParams p = shell_params(c, sd, q, nullptr, 0.0);
    int e = launch_shell_energy(c->precision, c->S.ref.N, p, s);
    if (e == 0) e = launch_sum_into(p.partial, sd.nsb, scale, acc, s);
    if (e != 0) throw Error(WDG_EHIP, std::string("shell energy launch: ") + hipGetErrorString(static_cast<hipError_t>(e)));
}

// y_next (optional): also write yn_a * (y_scale * y) + yn_b * qhat_out, with y the stage input
// (weight-adjusted inverse = identity only, where z is y itself up to the factor y_scale)
int adjoint_stage(wdg_ctx* c, const void* z, const void* y, const void* qhat_in, void* qhat_out, const void* q_fwd,
                  double* grad, double dt, hipStream_t s, void* y_next = nullptr, double yn_a = 0.0, double yn_b = 0.0,
                  double y_scale = 1.0) {
    const Setup& S = c->S;
    StageParams p{};
    p.q_in = z;
    p.q_out = qhat_out;
    p.res = const_cast<void*>(y);
    p.geo = c->geo.p;
    p.nbr = static_cast<const int*>(c->nbr.p);
    p.sigma = c->sigma.p;
    p.kappa = c->kappa.p;
    p.fmask = static_cast<const int*>(c->fmask.p);
    p.src_slot = static_cast<const int*>(c->src_slot.p);
    p.src = c->src.p;
    p.frags = c->frags.p;
    p.q_base = qhat_in;
    p.q_fwd = q_fwd;
    p.grad = grad;
    p.cub_w = static_cast<const double*>(c->cubw.p);
    p.Jk = static_cast<const double*>(c->Jk.p);
    p.nblk_pml = S.nblk_pml;
    p.nblk = S.nblk;
    p.pml0 = 0;
    p.npml = S.nblk_pml;
    p.int0 = S.nblk_pml;
    p.nint = S.nblk - S.nblk_pml;
    p.Nq = S.ref.Nq;
    p.read_res = 1;
    p.order_rev = c->next_order_rev();
    p.rk_a = 0.0;
    p.rk_b = 0.0;
    p.dt = dt;
    p.alpha = -S.flux_alpha;  // the upwind penalty changes sign in the adjoint
    p.src_g = 0.0;
    p.y_next = y_next;
    p.yn_a = yn_a;
    p.yn_b = yn_b;
    p.y_scale = y_scale;
    return launch_adjoint_mfma(c->precision, S.ref.N, p, s);
}

// d sigma_a / d theta at x for theta = (sigma_max xyz, L xyz, order), outer wall fixed.
void profile_derivatives(const PmlParams& pm, const double* x, double out[3][7]) {
    for (int a = 0; a < 3; ++a) {
        for (int t = 0; t < 7; ++t) out[a][t] = 0.0;
        const double d = std::max(0.0, std::max(x[a] - pm.hi[a], pm.lo[a] - x[a]));
        if (!(d > 0.0)) continue;
        const double r = d / pm.L[a], p = pm.order;
        const double rp = std::pow(r, p);
        out[a][a] = rp;
        out[a][3 + a] = pm.sigma_max[a] * p * std::pow(r, p - 1.0) * (1.0 - r) / pm.L[a];
        out[a][6] = pm.sigma_max[a] * rp * std::log(r);
    }
}

}  // namespace

extern "C" {

int32_t wdg_set_sigma_q(wdg_ctx* c, const double* sigma) {
    if (!c || !sigma) return WDG_EINVAL;
    if (c->pml_scheme != WDG_PML_WAA) return fail(c, WDG_ESTATE, "sigma at the cubature points is used by the weight-adjusted scheme only");
    return guarded(c, [&]() -> int {
        Setup& S = c->S;
        const size_t n = static_cast<size_t>(S.K) * S.ref.Nq * 3;
        for (int k = 0; k < S.K; ++k)
            for (size_t i = 0; i < static_cast<size_t>(S.ref.Nq) * 3; ++i) {
                const double v = sigma[static_cast<size_t>(k) * S.ref.Nq * 3 + i];
                if (!std::isfinite(v)) return fail(c, WDG_EINVAL, "sigma must be finite");
                if (!S.is_pml[k] && v != 0.0) return fail(c, WDG_EINVAL, "sigma must stay zero outside the PML elements");
            }
        S.sigma.assign(sigma, sigma + n);
        c->sigma_custom = true;
        if (!c->host_only) upload_coefficients(c);
        return WDG_OK;
    });
}

int32_t wdg_set_pml_profile(wdg_ctx* c, const double* sigma_max, const double* L, double order) {
    if (!c || !sigma_max || !L) return WDG_EINVAL;
    if (c->S.has_kappa) return fail(c, WDG_ESTATE, "profile parameters are re-sampled for kappa = 1 only");
    if (c->pml_scheme != WDG_PML_WAA) return fail(c, WDG_ESTATE, "sigma at the cubature points is used by the weight-adjusted scheme only");
    if (!(order >= 0.0) || !std::isfinite(order)) return fail(c, WDG_EINVAL, "profile order must be finite and >= 0");
    for (int d = 0; d < 3; ++d)
        if (!(L[d] > 0.0) || !(sigma_max[d] >= 0.0) || !std::isfinite(L[d]) || !std::isfinite(sigma_max[d]))
            return fail(c, WDG_EINVAL, "need L > 0 and sigma_max >= 0, finite");
    return guarded(c, [&]() -> int {
        Setup& S = c->S;
        PmlParams pm = S.pml;
        for (int d = 0; d < 3; ++d) {
            const double wall_lo = S.pml.lo[d] - S.pml.L[d], wall_hi = S.pml.hi[d] + S.pml.L[d];
            pm.lo[d] = wall_lo + L[d];
            pm.hi[d] = wall_hi - L[d];
            pm.L[d] = L[d];
            pm.sigma_max[d] = sigma_max[d];
        }
        pm.order = order;
        const int Nq = S.ref.Nq;
        std::vector<double> sig(static_cast<size_t>(S.K) * Nq * 3, 0.0);
        for (int k = 0; k < S.K; ++k)
            for (int q = 0; q < Nq; ++q)
                for (int d = 0; d < 3; ++d) {
                    const size_t i = (static_cast<size_t>(k) * Nq + q) * 3 + d;
                    sig[i] = pm.sigma_max[d] * profile_ratio(S.xq[i], pm.lo[d], pm.hi[d], pm.L[d], pm.order);
                    if (sig[i] != 0.0 && !S.is_pml[k])
                        return fail(c, WDG_EINVAL, "the layer would reach elements created outside it");
                }
        S.sigma.swap(sig);
        S.pml = pm;
        c->sigma_custom = false;
        if (!c->host_only) upload_coefficients(c);
        return WDG_OK;
    });
}

int32_t wdg_get_sigma_q(const wdg_ctx* c, double* sigma) {
    if (!c || !sigma) return WDG_EINVAL;
    std::copy(c->S.sigma.begin(), c->S.sigma.end(), sigma);
    return WDG_OK;
}

int32_t wdg_cubature_points(const wdg_ctx* c, double* xyz) {
    if (!c || !xyz) return WDG_EINVAL;
    std::copy(c->S.xq.begin(), c->S.xq.end(), xyz);
    return WDG_OK;
}

int32_t wdg_shell_energy(wdg_ctx* c, const wdg_shell* shell, double* out, void* hip_stream) {
    if (!c || !shell || !out) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return guarded(c, [&]() -> int {
        ShellDev sd;
        build_shell(c, *shell, sd);
        hip_check(hipMemsetAsync(c->scalar_out.p, 0, sizeof(double), s), "clear");
        shell_energy_into(c, sd, c->q[c->cur], 0.5, static_cast<double*>(c->scalar_out.p), s);
        hip_check(hipMemcpyAsync(out, c->scalar_out.p, sizeof(double), hipMemcpyDeviceToHost, s), "download");
        hip_check(hipStreamSynchronize(s), "sync");
        if (!std::isfinite(*out)) return fail(c, WDG_ENONFINITE, "shell energy is not finite");
        return WDG_OK;
    });
}

int32_t wdg_loss_gradient(wdg_ctx* c, double dt, int32_t nsteps, const wdg_shell* shell, int32_t checkpoint_interval,
                          double* loss, double* grad_sigma, double* grad_profile, void* hip_stream) {
    if (!c || !shell || !loss || nsteps < 0 || checkpoint_interval < 0 || !std::isfinite(dt)) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    const Setup& S = c->S;
    if (S.has_kappa) return fail(c, WDG_EINVAL, "the adjoint needs kappa = 1");
    if (c->has_dt_scale) return fail(c, WDG_EINVAL, "the adjoint needs one time step for all elements");
    if (c->pml_scheme != WDG_PML_WAA) return fail(c, WDG_EINVAL, "the adjoint is built for the weight-adjusted scheme");
    // kappa = 1 and a rule exact to degree 2N (checked at creation) make P_q a^-1 V_q the identity
    if (!c->waa_identity) return fail(c, WDG_EINVAL, "the adjoint needs P_q V_q = I");
    if (grad_profile && c->sigma_custom)
        return fail(c, WDG_ESTATE, "sigma was replaced point by point: no profile parameters describe it");
    if (!adjoint_supported(S.ref.N, S.ref.Nq, c->precision))
        return fail(c, WDG_EINVAL, "no adjoint kernel for this order, rule size and precision");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    TraceRange range("wdg_loss_gradient");
    return guarded(c, [&]() -> int {
        const int Nq = S.ref.Nq, B = S.B;
        const size_t bytes = static_cast<size_t>(c->state_elems) * c->rsize;
        const int C = checkpoint_interval > 0 ? checkpoint_interval
                                              : std::max(1, static_cast<int>(std::ceil(std::sqrt(static_cast<double>(nsteps)))));
        const int nseg = (nsteps + C - 1) / C;
        ShellDev sd;
        build_shell(c, *shell, sd);
        DevBuf acc, ckpt, stages, qh, y, rtmp, grad;
        int yc = 0;  // current half of y
        acc.alloc(sizeof(double));
        ckpt.alloc(static_cast<size_t>(nseg - 1) * bytes);  // the last segment keeps its stage inputs instead
        stages.alloc(static_cast<size_t>(5 * std::min(C, std::max(nsteps, 1)) + 1) * bytes);
        qh.alloc(2 * bytes);
        y.alloc(2 * bytes);
        rtmp.alloc(bytes);
        const size_t ngrad = static_cast<size_t>(std::max(S.nblk_pml, 1)) * 3 * Nq * B;
        grad.alloc(ngrad * sizeof(double));
        auto st = [&](int i) { return static_cast<char*>(stages.p) + static_cast<size_t>(i) * bytes; };
        auto qhb = [&](int i) { return static_cast<char*>(qh.p) + static_cast<size_t>(i) * bytes; };
        auto yb = [&](int i) { return static_cast<char*>(y.p) + static_cast<size_t>(i) * bytes; };
        hip_check(hipMemsetAsync(acc.p, 0, sizeof(double), s), "clear");

        // ---- forward sweep: the context's state advances; checkpoints and the loss.  The last segment's
        // stage inputs are written straight into the stage buffers, so the reverse sweep does not
        // recompute that segment (the same launches on the same inputs as a recomputation)
        const double t0 = c->t;
        const int last0 = (nseg - 1) * C;  // first step of the last segment
        for (int n = 0; n < nsteps; ++n) {
            TraceRange fstep("forward step");
            if (n < last0) {
                if (n % C == 0)
                    hip_check(hipMemcpyAsync(static_cast<char*>(ckpt.p) + static_cast<size_t>(n / C) * bytes, c->q[c->cur],
                                             bytes, hipMemcpyDeviceToDevice, s),
                              "checkpoint");
                for (int i = 0; i < 5; ++i) {
                    const int rc = launch_stage_on(c, c->q[c->cur], c->q[1 - c->cur], c->res, kRkA[i], kRkB[i], dt,
                                                   c->t + kRkC[i] * dt, i > 0, s);
                    if (rc != WDG_OK) return rc;
                    c->cur = 1 - c->cur;
                }
                c->t += dt;
                c->steps += 1;
                shell_energy_into(c, sd, c->q[c->cur], 0.5 * dt, static_cast<double*>(acc.p), s);
                continue;
            }
            const int j = n - last0;
            if (j == 0) hip_check(hipMemcpyAsync(st(0), c->q[c->cur], bytes, hipMemcpyDeviceToDevice, s), "checkpoint");
            for (int i = 0; i < 5; ++i) {
                const int rc = launch_stage_on(c, st(5 * j + i), st(5 * j + i + 1), c->res, kRkA[i], kRkB[i], dt,
                                               c->t + kRkC[i] * dt, i > 0, s);
                if (rc != WDG_OK) return rc;
            }
            c->t += dt;
            c->steps += 1;
            shell_energy_into(c, sd, st(5 * (j + 1)), 0.5 * dt, static_cast<double*>(acc.p), s);
        }
        if (nsteps > last0) {  // the final state back into the context's buffers, where stepping leaves it
            const int m = nsteps - last0;
            if ((5 * m) % 2) c->cur = 1 - c->cur;
            hip_check(hipMemcpyAsync(c->q[c->cur], st(5 * m), bytes, hipMemcpyDeviceToDevice, s), "final state");
        }

        // ---- adjoint sweep, segment by segment from the last
        hip_check(hipMemsetAsync(qh.p, 0, bytes, s), "clear");
        hip_check(hipMemsetAsync(grad.p, 0, ngrad * sizeof(double), s), "clear");
        int hc = 0;
        for (int seg = nseg - 1; seg >= 0; --seg) {
            TraceRange aseg("adjoint segment");
            const int n0 = seg * C, m = std::min(nsteps, n0 + C) - n0;
            // the last segment's stage inputs are already in the stage buffers (forward sweep)
            if (seg != nseg - 1)
                hip_check(hipMemcpyAsync(st(0), static_cast<char*>(ckpt.p) + static_cast<size_t>(seg) * bytes, bytes,
                                         hipMemcpyDeviceToDevice, s),
                          "restore");
            double t = t0 + n0 * dt;
            for (int jstep = 0; jstep < (seg == nseg - 1 ? 0 : m); ++jstep) {
                for (int i = 0; i < 5; ++i) {
                    const int rc = launch_stage_on(c, st(5 * jstep + i), st(5 * jstep + i + 1), rtmp.p, kRkA[i], kRkB[i], dt,
                                                   t + kRkC[i] * dt, i > 0, s);
                    if (rc != WDG_OK) return rc;
                }
                t += dt;
            }
            for (int jstep = m - 1; jstep >= 0; --jstep) {
                // dJ/dq_{n+1} of the step's loss term (M-weighted): dt P_q (chi V_q u)
                if (sd.nsb > 0) {
                    const ShellParams sp = shell_params(c, sd, st(5 * (jstep + 1)), qhb(hc), dt);
                    const int e = launch_shell_inject(c->precision, S.ref.N, sp, s);
                    if (e != 0) return fail(c, WDG_EHIP, "shell gradient launch");
                }
                // Stages reversed: y_i = A_{i+1} y_{i+1} + B_i q_hat (A_5 = 0), q_hat += dt L* y_i.  With
                // kappa = 1 the weight-adjusted inverse is the identity, so z = y: every stage takes its y
                // as input and writes the next stage's y (ping-pong halves); the first stage of the step,
                // y_4 = B_4 q_hat, reads q_hat with dt scaled by B_4 (L* and the sigma gradient are linear in y).
                for (int i = 4; i >= 0; --i) {
                    const void* in = i == 4 ? static_cast<const void*>(qhb(hc)) : static_cast<const void*>(yb(yc));
                    const double scale = i == 4 ? kRkB[4] : 1.0;
                    void* out = i > 0 ? yb(1 - yc) : nullptr;
                    const int e = adjoint_stage(c, in, in, qhb(hc), qhb(1 - hc), st(5 * jstep + i), static_cast<double*>(grad.p),
                                                dt * scale, s, out, i > 0 ? kRkA[i] : 0.0, i > 0 ? kRkB[i - 1] : 0.0, scale);
                    if (e != 0)
                        return fail(c, WDG_EHIP, std::string("adjoint launch: ") + hipGetErrorString(static_cast<hipError_t>(e)));
                    hc = 1 - hc;
                    if (i > 0) yc = 1 - yc;
                }
            }
        }

        // ---- results
        std::vector<double> g(ngrad);
        hip_check(hipMemcpyAsync(loss, acc.p, sizeof(double), hipMemcpyDeviceToHost, s), "download");
        hip_check(hipMemcpyAsync(g.data(), grad.p, ngrad * sizeof(double), hipMemcpyDeviceToHost, s), "download");
        hip_check(hipStreamSynchronize(s), "sync");
        if (!std::isfinite(*loss)) return fail(c, WDG_ENONFINITE, "loss is not finite");
        std::vector<double> gs(static_cast<size_t>(S.K) * Nq * 3, 0.0);
        for (int slot = 0; slot < S.nblk_pml * B; ++slot) {
            const int k = S.slot_elem[slot];
            if (k < 0) continue;
            const int blk = slot / B, lane = slot % B;
            for (int a = 0; a < 3; ++a)
                for (int q = 0; q < Nq; ++q)
                    gs[(static_cast<size_t>(k) * Nq + q) * 3 + a] = g[((static_cast<size_t>(blk) * 3 + a) * Nq + q) * B + lane];
        }
        if (grad_sigma) std::copy(gs.begin(), gs.end(), grad_sigma);
        if (grad_profile) {
            double acc7[7] = {0, 0, 0, 0, 0, 0, 0};
            double dsig[3][7];
            for (int k = 0; k < S.K; ++k) {
                if (!S.is_pml[k]) continue;
                for (int q = 0; q < Nq; ++q) {
                    profile_derivatives(S.pml, &S.xq[(static_cast<size_t>(k) * Nq + q) * 3], dsig);
                    for (int a = 0; a < 3; ++a)
                        for (int t = 0; t < 7; ++t) acc7[t] += gs[(static_cast<size_t>(k) * Nq + q) * 3 + a] * dsig[a][t];
                }
            }
            std::copy(acc7, acc7 + 7, grad_profile);
        }
        return WDG_OK;
    });
}

}  // extern "C"
