// Many independent simulations in one launch, captured stepping and the
// stage-kernel autotuner (C ABI part).
//
// Independent simulations share a context as one mesh with disjoint vertex
// sets (no face is shared, so no flux couples them).  Each keeps its own PML
// profile (wdg_set_sigma_profile) and its own stable time step (a per-element
// factor on dt, wdg_set_dt_scale); every element's arithmetic is independent
// of the other columns of its tile, so a simulation in a batch reproduces its
// standalone run bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <limits>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "context.hpp"

using namespace wdg;

namespace {

int launch_steps(wdg_ctx* c, double dt, int nsteps, hipStream_t s) {
    for (int n = 0; n < nsteps; ++n) {
        for (int i = 0; i < 5; ++i) {
            const int rc = launch_stage_on(c, c->q[c->cur], c->q[1 - c->cur], c->res, kRkA[i], kRkB[i], dt, c->t + kRkC[i] * dt,
                                           i > 0, s);
            if (rc != WDG_OK) return rc;
            c->cur = 1 - c->cur;
        }
        c->t += dt;
        c->steps += 1;
    }
    return WDG_OK;
}

// Autotune cache: the chosen (kernel, tiles) per device architecture, order, rule size, precision, PML
// scheme, kappa and mesh size class (blocks rounded to a power of two), in this process and, when the
// environment variable WDG_AUTOTUNE_CACHE names a file, in that file (one "key kernel tiles" line per
// entry, appended as entries are made).
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const wdg_ctx* c) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    int cls = 0;
    while ((1 << cls) < c->S.nblk) ++cls;
    std::ostringstream k;
    k << arch << "/N" << c->S.ref.N << "/q" << c->S.ref.Nq << "/" << (c->precision == WDG_FP64 ? "f64" : "f32") << "/s"
      << c->pml_scheme << "/k" << (c->S.has_kappa ? 1 : 0) << "/b" << cls;
    return k.str();
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("WDG_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string key;
    int kernel = 0, tiles = 0;
    while (f >> key >> kernel >> tiles)
        if ((kernel == WDG_KERNEL_SCALAR || kernel == WDG_KERNEL_MFMA) && (tiles == 1 || tiles == 2)) g_tune[key] = {kernel, tiles};
}

void tune_store_locked(const std::string& key, int kernel, int tiles) {
    g_tune[key] = {kernel, tiles};
    const char* path = std::getenv("WDG_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << kernel << " " << tiles << "\n";
}

}  // namespace

extern "C" {

int32_t wdg_autotune_cached(wdg_ctx* c, int32_t reps, void* hip_stream, int32_t* from_cache) {
    if (!c || reps < 1) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    const std::string key = tune_key(c);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_load_locked();
        const auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            const int kernel = it->second.first, tiles = it->second.second;
            const bool ok = kernel == WDG_KERNEL_SCALAR ||
                            (c->mfma_ok && mfma_tiles_fit(c->S.ref.N, c->S.ref.Nq, c->precision, tiles));
            if (ok) {
                c->kernel = kernel;
                c->tpw = kernel == WDG_KERNEL_MFMA ? tiles : c->tpw;
                c->drop_graph();
                if (from_cache) *from_cache = 1;
                return WDG_OK;
            }
        }
    }
    const int rc = wdg_autotune(c, reps, nullptr, hip_stream);
    if (rc != WDG_OK) return rc;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_store_locked(key, c->kernel, c->tpw);
    }
    if (from_cache) *from_cache = 0;
    return WDG_OK;
}

int32_t wdg_set_tiles(wdg_ctx* c, int32_t tiles) {
    if (!c) return WDG_EINVAL;
    if (tiles != 1 && tiles != 2) return fail(c, WDG_EINVAL, "tiles per workgroup must be 1 or 2");
    if (c->mfma_ok && !mfma_tiles_fit(c->S.ref.N, c->S.ref.Nq, c->precision, tiles))
        return fail(c, WDG_EINVAL, "this many tiles per workgroup need more LDS than a compute unit has");
    c->tpw = tiles;
    return WDG_OK;
}

int32_t wdg_set_step_groups(wdg_ctx* c, int32_t ngroups, const int32_t* group) {
    if (!c || ngroups < 0) return WDG_EINVAL;
    if (ngroups == 0 || !group) {
        c->drop_graph();
        c->groups.clear();
        return WDG_OK;
    }
    const Setup& S = c->S;
    if (!S.aligned) return fail(c, WDG_ESTATE, "step groups need a context created with WDG_ALIGN_COMPONENTS");
    return guarded(c, [&]() -> int {
        std::vector<int> cg(S.ncomp, -1);  // group of each component
        for (int k = 0; k < S.K; ++k) {
            const int g = group[k];
            if (g < 0 || g >= ngroups) return fail(c, WDG_EINVAL, "group index out of range");
            int& x = cg[S.comp[k]];
            if (x >= 0 && x != g) return fail(c, WDG_EINVAL, "a face-connected component spans two groups");
            x = g;
        }
        std::vector<std::array<int, 4>> out(ngroups, std::array<int, 4>{0, 0, 0, 0});
        std::vector<int> first(ngroups, -1), last(ngroups, -1);
        for (int cp = 0; cp < S.ncomp; ++cp) {
            const int g = cg[cp];
            if (first[g] < 0) first[g] = cp;
            else if (last[g] != cp - 1) return fail(c, WDG_EINVAL, "a group is not a run of consecutive components");
            last[g] = cp;
        }
        for (int g = 0; g < ngroups; ++g) {
            if (first[g] < 0) return fail(c, WDG_EINVAL, "an empty group");
            // blocks of the run in each class (components of a run are laid out one after another)
            int p0 = 0, p1 = 0, i0 = 0, i1 = 0;
            bool hp = false, hi = false;
            for (int cp = first[g]; cp <= last[g]; ++cp) {
                if (S.comp_pml1[cp] > S.comp_pml0[cp]) {
                    p0 = hp ? std::min(p0, S.comp_pml0[cp]) : S.comp_pml0[cp];
                    p1 = hp ? std::max(p1, S.comp_pml1[cp]) : S.comp_pml1[cp];
                    hp = true;
                }
                if (S.comp_int1[cp] > S.comp_int0[cp]) {
                    i0 = hi ? std::min(i0, S.comp_int0[cp]) : S.comp_int0[cp];
                    i1 = hi ? std::max(i1, S.comp_int1[cp]) : S.comp_int1[cp];
                    hi = true;
                }
            }
            out[g] = {p0, p1 - p0, hi ? i0 : S.nblk_pml, i1 - i0};
        }
        c->drop_graph();
        c->groups.swap(out);
        return WDG_OK;
    });
}

int32_t wdg_set_schedule(wdg_ctx* c, int32_t mode) {
    if (!c || (mode != WDG_SCHEDULE_FORWARD && mode != WDG_SCHEDULE_REVERSED && mode != WDG_SCHEDULE_ALTERNATING))
        return WDG_EINVAL;
    c->drop_graph();
    c->schedule = mode;
    c->sweep_count = 0;
    return WDG_OK;
}

int32_t wdg_set_waa_shortcut(wdg_ctx* c, int32_t on) {
    if (!c) return WDG_EINVAL;
    if (on && !c->waa_identity)
        return fail(c, WDG_EINVAL, "the weight-adjusted inverse is not the identity here (kappa != 1 or P_q V_q != I)");
    c->waa_skip = on != 0;
    return WDG_OK;
}

int32_t wdg_set_dt_scale(wdg_ctx* c, const double* scale) {
    if (!c) return WDG_EINVAL;
    if (c->host_only) return fail(c, WDG_ESTATE, "host-only context");
    return guarded(c, [&]() -> int {
        const Setup& S = c->S;
        c->drop_graph();
        if (!scale) {
            c->has_dt_scale = false;
            c->dt_scale.alloc(0);
            return WDG_OK;
        }
        std::vector<double> d(static_cast<size_t>(S.nblk) * S.B, 1.0);
        for (int k = 0; k < S.K; ++k) {
            if (!(scale[k] > 0.0) || !std::isfinite(scale[k])) return fail(c, WDG_EINVAL, "dt scale must be positive and finite");
            d[S.perm[k]] = scale[k];
        }
        c->dt_scale.upload(d.data(), d.size() * sizeof(double));
        c->has_dt_scale = true;
        return WDG_OK;
    });
}

int32_t wdg_set_sigma_profile(wdg_ctx* c, const int32_t* group, int32_t ngroups, const double* sigma_max, const double* order) {
    if (!c || !group || ngroups <= 0 || !sigma_max || !order) return WDG_EINVAL;
    if (c->pml_scheme != WDG_PML_WAA) return fail(c, WDG_ESTATE, "per-group profiles are used by the weight-adjusted scheme only");
    return guarded(c, [&]() -> int {
        Setup& S = c->S;
        if (S.has_kappa) return fail(c, WDG_EINVAL, "per-group profiles need kappa = 1");
        for (int g = 0; g < ngroups; ++g) {
            if (!(order[g] >= 0.0)) return fail(c, WDG_EINVAL, "profile order must be >= 0");
            for (int d = 0; d < 3; ++d)
                if (!(sigma_max[3 * g + d] >= 0.0)) return fail(c, WDG_EINVAL, "sigma_max must be >= 0");
        }
        const int Nq = S.ref.Nq;
        std::vector<double> sig(static_cast<size_t>(S.K) * Nq * 3, 0.0);
        for (int k = 0; k < S.K; ++k) {
            const int g = group[k];
            if (g < 0 || g >= ngroups) return fail(c, WDG_EINVAL, "group index out of range");
            if (!S.is_pml[k]) continue;
            for (int q = 0; q < Nq; ++q)
                for (int d = 0; d < 3; ++d) {
                    const size_t i = (static_cast<size_t>(k) * Nq + q) * 3 + d;
                    sig[i] = sigma_max[3 * g + d] *
                             profile_ratio(S.xq[i], S.pml.lo[d], S.pml.hi[d], S.pml.L[d], order[g]);
                }
        }
        S.sigma.swap(sig);
        c->sigma_custom = true;
        if (!c->host_only) upload_coefficients(c);
        return WDG_OK;
    });
}

int32_t wdg_step_graph(wdg_ctx* c, double dt, int32_t nsteps, void* hip_stream) {
    if (!c || nsteps < 0 || !std::isfinite(dt)) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    if (!hip_stream) return fail(c, WDG_EINVAL, "graph stepping needs a non-null stream");
    if (c->has_src) return fail(c, WDG_EINVAL, "graph stepping needs no source (its amplitude changes every stage)");
    if (c->nprobe > 0) return fail(c, WDG_EINVAL, "graph stepping needs no probes");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    TraceRange range("wdg_step_graph");
    return guarded(c, [&]() -> int {
        const int pairs = nsteps / 2;
        if (pairs > 0) {
            const bool same = c->graph && c->graph_dt == dt && c->graph_cur == c->cur && c->graph_kernel == c->kernel &&
                              c->graph_tpw == c->tpw && c->graph_scheme == c->pml_scheme && c->graph_skip == (c->waa_skip ? 1 : 0) && c->graph_bufs[0] == c->q[0] && c->graph_bufs[1] == c->q[1] &&
                              c->graph_bufs[2] == c->res;
            if (!same) {
                c->drop_graph();
                // Capture two steps (ten stage launches): the buffer roles are
                // back where they started, so one graph serves every pair.
                const int cur0 = c->cur;
                const double t0 = c->t;
                const int64_t s0 = c->steps;
                hipGraph_t g = nullptr;
                hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
                int rc = WDG_OK;
                if (c->groups.empty()) {
                    rc = launch_steps(c, dt, 2, s);
                } else {
                    // group after group, both steps on that group's blocks (its fields stay in the
                    // last-level cache over the ten stages); each group starts from the same buffers
                    for (size_t gi = 0; gi < c->groups.size() && rc == WDG_OK; ++gi) {
                        c->cur = cur0;
                        c->t = t0;
                        c->range = c->groups[gi];
                        c->range_on = true;
                        rc = launch_steps(c, dt, 2, s);
                        c->range_on = false;
                    }
                }
                const hipError_t ec = hipStreamEndCapture(s, &g);
                c->cur = cur0;
                c->t = t0;
                c->steps = s0;
                if (rc != WDG_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return rc;
                }
                hip_check(ec, "end capture");
                hipGraphExec_t ex = nullptr;
                const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                hip_check(ei, "graph instantiate");
                c->graph = ex;
                c->graph_dt = dt;
                c->graph_cur = c->cur;
                c->graph_kernel = c->kernel;
                c->graph_tpw = c->tpw;
                c->graph_skip = c->waa_skip ? 1 : 0;
                c->graph_scheme = c->pml_scheme;
                c->graph_bufs[0] = c->q[0];
                c->graph_bufs[1] = c->q[1];
                c->graph_bufs[2] = c->res;
            }
            for (int i = 0; i < pairs; ++i) hip_check(hipGraphLaunch(c->graph, s), "graph launch");
            // the clock advances as eager stepping advances it, one dt at a time
            for (int i = 0; i < 2 * pairs; ++i) c->t += dt;
            c->steps += 2 * pairs;
        }
        if (nsteps % 2) return launch_steps(c, dt, 1, s);
        return WDG_OK;
    });
}

int32_t wdg_autotune(wdg_ctx* c, int32_t reps, double* times_us, void* hip_stream) {
    if (!c || reps < 1) return WDG_EINVAL;
    if (int e = check_state(c)) return e;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return guarded(c, [&]() -> int {
        struct Cand {
            int kernel, tpw;
        };
        const Cand cands[3] = {{WDG_KERNEL_SCALAR, 2}, {WDG_KERNEL_MFMA, 1}, {WDG_KERNEL_MFMA, 2}};
        double best = std::numeric_limits<double>::infinity();
        int best_i = -1;
        const int kernel0 = c->kernel, tpw0 = c->tpw;
        hipEvent_t a = nullptr, b = nullptr;
        hip_check(hipEventCreate(&a), "event");
        hip_check(hipEventCreate(&b), "event");
        int rc = WDG_OK;
        for (int i = 0; i < 3 && rc == WDG_OK; ++i) {
            double t_us = -1.0;
            if (cands[i].kernel != WDG_KERNEL_MFMA ||
                (c->mfma_ok && mfma_tiles_fit(c->S.ref.N, c->S.ref.Nq, c->precision, cands[i].tpw))) {
                c->kernel = cands[i].kernel;
                c->tpw = cands[i].tpw;
                // a stage as in the middle of a step: reads and writes the residual,
                // writes the spare field buffer; the current fields are untouched
                auto stage = [&]() {
                    return launch_stage_on(c, c->q[c->cur], c->q[1 - c->cur], c->res, kRkA[1], kRkB[1], 1e-30, c->t, true, s);
                };
                rc = stage();  // warm-up
                float best_ms = std::numeric_limits<float>::infinity();
                for (int trial = 0; trial < 3 && rc == WDG_OK; ++trial) {
                    hip_check(hipEventRecord(a, s), "event");
                    for (int r = 0; r < reps && rc == WDG_OK; ++r) rc = stage();
                    hip_check(hipEventRecord(b, s), "event");
                    hip_check(hipEventSynchronize(b), "event");
                    float ms = 0.0f;
                    hip_check(hipEventElapsedTime(&ms, a, b), "event");
                    best_ms = std::min(best_ms, ms);
                }
                t_us = 1e3 * best_ms / reps;
                if (rc == WDG_OK && t_us < best) {
                    best = t_us;
                    best_i = i;
                }
            }
            if (times_us) times_us[i] = t_us;
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (rc != WDG_OK || best_i < 0) {
            c->kernel = kernel0;
            c->tpw = tpw0;
            return rc != WDG_OK ? rc : fail(c, WDG_EHIP, "no stage kernel ran");
        }
        c->kernel = cands[best_i].kernel;
        c->tpw = cands[best_i].tpw;
        return WDG_OK;
    });
}

}  // extern "C"
