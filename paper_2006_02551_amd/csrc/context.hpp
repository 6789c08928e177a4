// Library context shared by the C ABI translation units (api.cpp, adjoint.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wdg.h"
#include "device.hpp"
#include "host.hpp"
#include "trace.hpp"

namespace wdg {

// LSERK4 coefficients (Carpenter & Kennedy 1994, five-stage 2N-storage,
// fourth order), as the published rationals.
inline constexpr double kRkA[5] = {0.0,
                                   -567301805773.0 / 1357537059087.0,
                                   -2404267990393.0 / 2016746695238.0,
                                   -3550918686646.0 / 2091501179385.0,
                                   -1275806237668.0 / 842570457699.0};
inline constexpr double kRkB[5] = {1432997174477.0 / 9575080441755.0,
                                   5161836677717.0 / 13612068292357.0,
                                   1720146321549.0 / 2090206949498.0,
                                   3134564353537.0 / 4481467310338.0,
                                   2277821191437.0 / 14882151754819.0};
inline constexpr double kRkC[5] = {0.0,
                                   1432997174477.0 / 9575080441755.0,
                                   2526269341429.0 / 6820363962896.0,
                                   2006345519317.0 / 3224310063776.0,
                                   2802321613138.0 / 2924317926251.0};

void hip_check(hipError_t e, const char* what);

// Device allocation owned by the library.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    void alloc(size_t n) {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = n;
        if (n == 0) return;
        const hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error(WDG_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
    }
    void upload(const void* src, size_t n) {
        alloc(n);
        if (n == 0) return;
        hip_check(hipMemcpy(p, src, n, hipMemcpyHostToDevice), "hipMemcpy");
    }
};

// FP64 host values as the context's precision (raw bytes).
std::vector<unsigned char> to_real(const std::vector<double>& v, int precision);

}  // namespace wdg

struct wdg_ctx {
    wdg::Setup S;
    int precision = WDG_FP64;
    bool host_only = false;
    std::string err;
    int device = 0;
    size_t rsize = 8;
    int64_t state_elems = 0;
    // device setup
    wdg::DevBuf geo, nbr, sigma, kappa, ops, fmask, Jk, Mref, partial, scalar_out, cubw;
    wdg::DevBuf src_slot, src;
    wdg::DevBuf frags;
    bool mfma_ok = false;
    bool waa_identity = false;  // kappa = 1 and P_q V_q = I to rounding
    bool waa_skip = false;      // skip the weight-adjusted inverse (only where waa_identity holds; opt-in)
    int schedule = WDG_SCHEDULE_ALTERNATING;  // order in which workgroups take the tiles (wdg_set_schedule)
    uint64_t sweep_count = 0;                  // stage launches made with the alternating schedule
    // reversed order for the next stage launch (advances the alternating schedule)
    int next_order_rev() {
        if (schedule == WDG_SCHEDULE_ALTERNATING) return static_cast<int>(sweep_count++ & 1);
        return schedule == WDG_SCHEDULE_REVERSED ? 1 : 0;
    }
    // step groups (aligned layouts only): per group [pml0, npml, int0, nint] block ranges; stage launches
    // cover range while range_on
    std::vector<std::array<int, 4>> groups;
    bool range_on = false;
    std::array<int, 4> range{};
    int kernel = WDG_KERNEL_SCALAR;
    int tpw = 2;  // tiles per workgroup of the matrix-core kernel
    // PML scheme (WDG_PML_*) and its per-element data: the direct scheme's stored
    // matrices or the element-constant coefficients (empty for the weight-adjusted scheme)
    int pml_scheme = WDG_PML_WAA;
    wdg::DevBuf pml_mats, pml_work;
    bool sigma_custom = false;  // sigma at the cubature points no longer follows the method's profile
    // per-element factor on dt (independent simulations sharing one launch)
    wdg::DevBuf dt_scale;
    bool has_dt_scale = false;
    // captured two-step graph of wdg_step_graph and what it was captured for
    hipGraphExec_t graph = nullptr;
    double graph_dt = 0.0;
    int graph_cur = -1, graph_kernel = -1, graph_tpw = -1, graph_scheme = -1, graph_skip = -1;
    void* graph_bufs[3] = {nullptr, nullptr, nullptr};
    ~wdg_ctx() { drop_graph(); }
    // A captured graph holds the device addresses of every buffer a stage reads;
    // whatever reallocates one of them drops the graph.
    void drop_graph() {
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
    }
    bool has_src = false;
    wdg_dipole dip{};
    // probes
    int nprobe = 0, probe_cap = 0, probe_rows = 0;
    wdg::DevBuf probe_slot, probe_w, probe_buf;
    // state
    void* q[2] = {nullptr, nullptr};
    void* res = nullptr;
    int cur = 0;
    double t = 0.0;
    int64_t steps = 0;
    size_t off_DrT = 0, off_DsT = 0, off_DtT = 0, off_LIFTT = 0, off_Vq = 0, off_PqT = 0;
};

namespace wdg {

int fail(wdg_ctx* ctx, int code, const std::string& msg);

template <typename F>
int guarded(wdg_ctx* ctx, F&& fn) {
    try {
        return fn();
    } catch (const Error& e) {
        return fail(ctx, e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(ctx, WDG_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(ctx, WDG_EINVAL, e.what());
    }
}

inline int64_t eh_words(const Setup& S) { return static_cast<int64_t>(6) * S.ref.Np * S.B; }
// largest E,H part (words) that 32-bit signed neighbour offsets can address
constexpr int64_t kMaxEhWords = 2147483647;

// Offset of (user element k, canonical component c, node i) in the blocked buffer, or -1.
int64_t state_index(const Setup& S, int k, int c, int i);

// Address of operator `off_words` words into the packed operator buffer.
inline const char* cptr(const DevBuf& b, size_t off_words, size_t rsize) {
    return static_cast<const char*>(b.p) + off_words * rsize;
}

// One Runge-Kutta stage of the forward scheme: res <- rk_a res + dt rhs(q_in, t),
// q_out <- q_in + rk_b res.
int launch_stage_on(wdg_ctx* c, const void* qin, void* qout, void* res, double rk_a, double rk_b, double dt, double t,
                    bool read_res, hipStream_t stream);

int check_state(wdg_ctx* c);

// Uploads sigma (and kappa) at the cubature points of the PML blocks from S.
void upload_coefficients(wdg_ctx* c);

// Device address of the allocation-free readout's scratch array on `device` (the current device),
// looked up once per device; returns a hipError_t (0 on success).
int noalloc_setup(int device);

}  // namespace wdg
