// Device-side parameter blocks and launchers shared by the C ABI and the
// kernels.  All pointers are device pointers.
//
// Blocked device layout (B = 64 element slots per block, PML blocks first):
//   fields   [nblk][6][Np][B]       E, H        then
//            [nblk_pml][6][Np][B]   P^E, P^H    (one buffer = both parts)
//   geometry [nblk][25][B]          rx ry rz sx sy sz tx ty tz, then per face
//                                   nx ny nz Fscale
//   nbr      [nblk][4 Nfp][B]       offset of the neighbour's trace value of
//                                   component 0 inside the E,H part, or the
//                                   bitwise complement of the own offset at a
//                                   PEC wall
//   sigma    [nblk_pml][3][Nq][B]   (kappa likewise when it is not one)
//   PML terms of the other schemes (scalar-operand kernel only):
//     direct            [nblk_pml][3 axes][5][Np][Np][B]  per element and axis u the
//                       products (M^a)^-1 M_k, (M^a)^-1 M^b, (M^a)^-1 M^c,
//                       M_k^-1 M^{1/kappa}, M_k^-1 M^d of the weighted mass
//                       matrices of eq. (15) (row i, column j)
//     element-constant  [nblk_pml][6][B]  sigma_x sigma_y sigma_z kappa_x kappa_y kappa_z
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wdg {

constexpr int kBlock = 64;   // element slots per block (one wavefront)
constexpr int kGeo = 25;     // geometry words per element slot
constexpr int kThreads = 6 * kBlock;  // one wavefront per field component
constexpr int kMfmaThreads = 6 * 64;  // MFMA kernel: one wavefront per component of a 16-element tile

// How the PML terms of eqs. (10)-(13) are evaluated (the values match WDG_PML_* of the C ABI).
enum PmlMode : int { kPmlWaa = 0, kPmlDirect = 1, kPmlConstant = 2 };
constexpr int kDirectMats = 5;  // stored products per element and axis

// MFMA operand fragments.  An operator with `rows` rows is cut into tiles of
// 16 rows; for every tile t and k-step s (4 columns) there is one fragment.
//
// FP32 (16x16x4 product): a full tile's fragment is 64 words, lane l holding
//   Op[16 t + 4 (r % 4) + r / 4][4 s + l / 16],  r = l % 16,
// so that register v of lane group g of a product holds row 16 t + 4 v + g.
// Stored compact, the last tile keeps only its m valid rows: 4 m words
// Op[16 t + i][4 s + k] at k m + i; lane l reads word (l / 16) m + min(i, m - 1)
// (rows past m repeat a valid row; the kernels never use those output rows).
//
// FP64 (four-block 4x4x4 products, one per result register v = rows 4v..4v+3
// of the tile): a full tile's fragment is 64 words, word 16 k + 4 i + v holding
//   Op[16 t + 4 v + i][4 s + k];
// lane l = 16 k + 4 b + i (b = column block) reads the four words 16 k + 4 i + v.
// Stored compact, the last tile keeps only its nv = ceil(m / 4) leading
// registers: 16 nv words, word 4 nv k + nv i + v (rows past m are zero).
constexpr int frag_words(int rows, int tiles, int ksteps, bool compact, bool f64) {
    const int m = rows - 16 * (tiles - 1);
    const int last = f64 ? 16 * ((m + 3) / 4) : 4 * m;
    return compact ? ((tiles - 1) * 64 + last) * ksteps : tiles * 64 * ksteps;
}
// Position `bid` of a launch over n0 + n1 work items (n0 of a first range starting at base0, n1 of a second
// starting at base1), mapped so that each of the eight XCDs (consecutive workgroup IDs go to consecutive
// XCDs) walks a contiguous run of items inside each range: neighbour traces then tend to hit its own L2.
__device__ __forceinline__ int remap_range(int bid, int base0, int n0, int base1, int n1) {
    int base = base0, n = n0, j = bid;
    if (bid >= n0) {
        base = base1;
        n = n1;
        j = bid - n0;
    }
    const int x = j & 7, i = j >> 3;
    const int q = n >> 3, r = n & 7;
    return base + x * q + (x < r ? x : r) + i;
}

// Number of 1 KiB chunks that hold nwords fragment words.
constexpr int frag_chunks(int nwords, int word_bytes) { return (nwords * word_bytes + 1023) / 1024; }

struct StageParams {
    const void* q_in;
    void* q_out;
    void* res;
    const void* geo;
    const int* nbr;
    const void* sigma;
    const void* kappa;
    const void* DrT;    // [Np][Np], DrT[j][i] = Dr[i][j]
    const void* DsT;
    const void* DtT;
    const void* LIFTT;  // [4 Nfp][Np]
    const void* Vq;     // [Nq][Np]
    const void* PqT;    // [Nq][Np], PqT[q][i] = Pq[i][q]
    const int* fmask;   // [4][Nfp]
    const int* src_slot;  // [nblk] source slot of a block or -1
    const void* src;      // [nslot][3][Np][B] J direction times spatial factor
    const void* frags;    // MFMA kernel: operator A fragments (V_q, P_q, D_r, D_s, D_t, LIFT)
    // adjoint stage only
    const void* q_base;   // running adjoint (the update's base)
    const void* q_fwd;    // forward stage input (for the sigma gradient)
    double* grad;         // [nblk_pml][3][Nq][B] sigma gradient accumulator (FP64)
    const double* cub_w;  // [Nq] cubature weights
    const double* Jk;     // [nblk][B] Jacobians
    const double* dt_scale;  // [nblk][B] per-element factor on dt, or null (uniform dt)
    // adjoint stage, weight-adjusted inverse = identity: also write the next stage's adjoint
    // y_next = yn_a * (y_scale * y) + yn_b * q_hat_out (null: not written); y is this stage's
    // input (q_in / res), given as y / y_scale
    void* y_next;
    double yn_a, yn_b, y_scale;
    const void* pml_mats;    // direct matrices or element-constant coefficients (see the layout above)
    void* pml_work;          // direct scheme: [nblk_pml][6][Np][B] vacuum right-hand side of the PML blocks
    int nblk_pml, nblk, Nq;
    // 1 when the caller asked to skip the weight-adjusted inverse where it is the identity (kappa = 1
    // and P_q V_q = I, a rule exact to degree 2N: a = 1 makes P_q a^-1 V_q = I); 0 (the default)
    // applies P_q a^-1 V_q on every PML element
    int waa_skip;
    int read_res;         // 0 when the Runge-Kutta coefficient A is zero
    int order_rev;        // 1: workgroups take their tiles / blocks in reversed order (wdg_set_schedule)
    // blocks this launch covers: [pml0, pml0 + npml) of the PML class and [int0, int0 + nint) of the vacuum
    // class (every block unless a launch is restricted to a group of independent simulations)
    int pml0, npml, int0, nint;
    double rk_a, rk_b, dt, src_g, alpha;
};

// Shell-energy loss and its gradient on the blocks holding shell points.
struct ShellParams {
    const void* q;        // state the energy is taken of
    void* q_hat;          // running adjoint (gradient injection)
    const int* blocks;    // [nsb] block of each shell block
    const void* chi;      // [nsb][Nq][B] shell indicator at the cubature points
    const double* Jk;     // [nblk][B]
    const double* cub_w;  // [Nq]
    const void* Vq;       // [Nq][Np]
    const void* PqT;      // [Nq][Np]
    double* partial;      // [nsb]
    int nsb, nblk, Nq;
    double dt;
};

struct ProbeParams {
    const void* q;
    const int* slot;       // [n] element slot of each probe
    const double* w;       // [n][Np] Lagrange weights
    double* out;           // [n][6] destination row
    int n;
};

struct EnergyParams {
    const void* q;
    const double* J;      // [nblk][B]
    const double* M;      // [Np][Np]
    double* partial;      // [nblk]
    int nblk;
};

// Launchers (kernels.hip, kernels_mfma.hip); return hipError_t as int.
// pml_mode: PmlMode; the direct and element-constant schemes ignore has_kappa (kappa is in their data).
int launch_stage(int precision, int N, bool has_kappa, int pml_mode, const StageParams& p, hipStream_t s);
// tpw: 16-element tiles per workgroup of the matrix-core kernel (1 or 2).
int launch_stage_mfma(int precision, int N, bool has_kappa, int tpw, int pml_mode, const StageParams& p, hipStream_t s);
// The direct scheme's second launch (stored products and update of the PML blocks), after a stage
// kernel in direct mode has written their vacuum right-hand side to p.pml_work.
int launch_direct_apply(int precision, int N, const StageParams& p, hipStream_t s);
// Adjoint stage on the matrix cores (kappa = 1; same (N, N_q) support as the forward).
int launch_adjoint_mfma(int precision, int N, const StageParams& p, hipStream_t s);
bool mfma_supported(int N, int Nq, int precision);
// whether the matrix-core kernel with tpw tiles per workgroup fits in a compute unit's LDS
bool mfma_tiles_fit(int N, int Nq, int precision, int tpw);
bool adjoint_supported(int N, int Nq, int precision);
int launch_probe(int precision, int N, const ProbeParams& p, hipStream_t s);
// partial[sb] = sum over the block's slots of J w_q chi (V_q u)^2 over the six E,H components
int launch_shell_energy(int precision, int N, const ShellParams& p, hipStream_t s);
// *acc += scale * sum(partial[0..n)) in a fixed order (one workgroup)
int launch_sum_into(const double* partial, int n, double scale, double* acc, hipStream_t s);
// q_hat += dt P_q (chi V_q u) for the six E,H components on the shell blocks
int launch_shell_inject(int precision, int N, const ShellParams& p, hipStream_t s);
int launch_energy(int precision, int N, const EnergyParams& p, double* out, hipStream_t s);

}  // namespace wdg
