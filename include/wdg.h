/*
 * wdg.h -- C ABI of the weight-adjusted smoothly-varying SC-PML DGTD library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library advances the semi-discrete Maxwell system with a stretched-
 * coordinate PML, eqs. (26)-(29) of Chen, Ozakin, Ahmed, Bagci,
 * "A Memory-efficient Implementation of Perfectly Matched Layer with
 * Smoothly-varying Coefficients in Discontinuous Galerkin Time-Domain Method"
 * (Sec. II-A), on affine tetrahedra with nodal Lagrange elements of order N,
 * the upwind curl operator of eqs. (15)-(17), the weight-adjusted inverse mass
 * of eq. (21) and the fused operators of eqs. (22)-(25), integrated in time by
 * the five-stage fourth-order low-storage Runge-Kutta scheme of Carpenter and
 * Kennedy (the paper leaves the integrator open).
 *
 * Conventions (fixed; they define the canonical user layout):
 *  - units are normalised: eps0 = mu0 = c = 1, vacuum inside elements;
 *  - reference tetrahedron v0=(-1,-1,-1), v1=(1,-1,-1), v2=(-1,1,-1),
 *    v3=(-1,-1,1); an element maps v_i to its i-th vertex; tetrahedra with
 *    negative orientation get their last two vertices swapped;
 *  - nodes: equispaced lattice r=-1+2a/N, s=-1+2b/N, t=-1+2c/N with
 *    a+b+c <= N, ordered c outermost, then b, then a;
 *  - canonical field array: double [K][12][Np] in user element order with
 *    components Ex Ey Ez Hx Hy Hz PEx PEy PEz PHx PHy PHz; the auxiliary
 *    components exist only in PML elements (ignored on set, zero on get);
 *  - a mesh face without a neighbour is a perfect electric conductor wall;
 *  - PML profile per axis u: with d_u the distance from the interface box
 *    [pml_lo, pml_hi] into the layer, sigma_u = sigma_max_u (d_u/L_u)^p and
 *    kappa_u = 1 + (kappa_max - 1)(d_u/L_u)^p (p = 0 means a step);
 *    an element is a PML element when sigma or kappa differ from vacuum at
 *    any of its cubature points.
 *
 * All functions return WDG_OK (0) or a negative error code; no C++ exception
 * crosses this boundary.  A context is not thread-safe: use one per host
 * thread and stream.  Inputs passed by pointer are copied unless stated.
 */
#ifndef WDG_H
#define WDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WDG_OK 0
#define WDG_EINVAL (-1)     /* bad argument (null pointer, size, order, rule) */
#define WDG_EMESH (-2)      /* degenerate tetrahedron, non-manifold or non-conforming face */
#define WDG_ENOMEM (-3)     /* host or device allocation failed */
#define WDG_EHIP (-4)       /* HIP runtime error (message in wdg_last_error) */
#define WDG_ESTATE (-5)     /* state buffers not bound, or a host-only context */
#define WDG_EPROBE (-6)     /* probe point outside the mesh, or probe buffer full */
#define WDG_ENONFINITE (-7) /* energy readout is not finite */

#define WDG_FP64 0
#define WDG_FP32 1

/* wdg_method.flags */
#define WDG_HOST_ONLY 1 /* build the host-side setup only: no device memory, no stepping */
/* start every face-connected component of the mesh (an independent simulation of a batch) at a block
 * boundary of each element class, so that stages can be launched per group of components
 * (wdg_set_step_groups); costs up to 63 padding slots per component and class */
#define WDG_ALIGN_COMPONENTS 2

typedef struct wdg_ctx wdg_ctx;

/* Tetrahedral mesh.  vxyz: double [nv][3]; etov: int32 [K][4] (0-based).
 * vertex_id: NULL, or int32 [nv] naming for every vertex the vertex it stands
 * for in the face connectivity (periodic meshes: a vertex on the upper face of a
 * periodic box identified with its image on the lower face).  Faces are matched
 * on identified vertex triples; geometry uses the coordinates as given.  A face
 * with no partner is a PEC wall.  The identification must keep the four vertices
 * of every element distinct (WDG_EMESH otherwise). */
typedef struct wdg_mesh {
    int32_t nv;
    const double* vxyz;
    int32_t K;
    const int32_t* etov;
    const int32_t* vertex_id;
} wdg_mesh;

/* Discretisation and PML parameters.
 * N: polynomial order, 1..4.  cub_rst: double [nq][3] reference coordinates,
 * cub_w: double [nq] weights of a cubature rule on the reference tetrahedron
 * that is exact to degree >= 2N (eqs. (19)-(20); nq <= 128).
 * flux_alpha: 1 upwind, 0 central.  precision: WDG_FP64 or WDG_FP32 (the
 * stepping arithmetic and state; setup is always FP64). */
typedef struct wdg_method {
    int32_t N;
    int32_t nq;
    const double* cub_rst;
    const double* cub_w;
    double flux_alpha;
    int32_t precision;
    int32_t flags;
    double pml_lo[3];
    double pml_hi[3];
    double pml_L[3];
    double sigma_max[3];
    double profile_order;
    double kappa_max;
} wdg_method;

typedef struct wdg_dims_t {
    int32_t K, K_pml, N, Np, Nfp, Nq;
    int32_t block;          /* elements per element block (device layout) */
    int32_t nblk_pml, nblk; /* PML blocks come first */
    int32_t precision;
    int32_t has_kappa;
    int64_t state_bytes; /* bytes of each of the three state buffers */
    double dt_unit;      /* 1 / ((N+1)^2 max_{k,f} Fscale_{k,f}); dt = cfl * dt_unit */
    double time;         /* current simulation time */
    int64_t steps;       /* steps taken since creation / last set_fields */
    int32_t kernel;      /* active stage-kernel variant (WDG_KERNEL_*) */
    int32_t tiles;       /* 16-element tiles per workgroup of the matrix-core kernel (1 or 2) */
    int32_t pml_scheme;  /* active PML scheme (WDG_PML_*) */
} wdg_dims_t;

/* Gaussian-modulated dipole current, added to dE/dt as -J:
 * J(x,t) = amplitude sin(2 pi f0 (t - t0)) exp(-((t - t0)/tau)^2)
 *          exp(-|x - center|^2 / width^2) direction.
 * Nodes where the spatial factor is below 1e-16 are left out. */
typedef struct wdg_dipole {
    double amplitude, f0, t0, tau;
    double center[3];
    double width;
    double direction[3];
} wdg_dipole;

/* Memory accounting (bytes), Sec. II-B: the direct method stores
 * 15 N_p^2 words per PML element, the weight-adjusted one 15 N_q words per PML
 * element plus 2 N_p N_q shared words; this library stores sigma (and kappa)
 * at the cubature points, 3 (6) N_q words per PML element. */
typedef struct wdg_mem_t {
    int64_t state;           /* three state buffers (caller-owned) */
    int64_t geometry;        /* metric terms, normals, Fscale, Jacobians */
    int64_t connectivity;    /* face-node neighbour map */
    int64_t coefficients;    /* sigma/kappa at cubature points */
    int64_t operators;       /* reference operators */
    int64_t paper_direct;    /* 15 N_p^2 K_pml words of the direct method */
    int64_t paper_waa;       /* 15 N_q K_pml + 2 N_p N_q words of the paper's WAA storage */
    int64_t scheme_data;     /* device bytes of the direct scheme's matrices or the element-constant
                                coefficients (0 for the weight-adjusted scheme) */
} wdg_mem_t;

/* Version: major*10000 + minor*100 + patch. */
int32_t wdg_version(void);

/* Message for an error code. */
const char* wdg_error_string(int32_t code);

/* Last error message of a context (or of the last failed wdg_create if ctx is NULL). */
const char* wdg_last_error(const wdg_ctx* ctx);

/* Builds the reference operators (eqs. (14)-(21)), geometry, face matching,
 * element classification and device layout; uploads them to the current HIP
 * device unless WDG_HOST_ONLY.  The mesh and method arrays are copied.
 * WDG_EINVAL if the E,H part of the state (nblk x 6 x N_p x 64 words) exceeds
 * 2^31 - 1 words, the reach of the 32-bit neighbour offsets (about 17.9M
 * tetrahedra at N = 3, 10.2M at N = 4); a larger mesh is split over devices. */
int32_t wdg_create(const wdg_mesh* mesh, const wdg_method* method, wdg_ctx** out);

/* Releases everything the library allocated.  Bound state buffers are not freed. */
void wdg_destroy(wdg_ctx* ctx);

int32_t wdg_get_dims(const wdg_ctx* ctx, wdg_dims_t* out);

/* Binds three caller-owned device buffers of dims.state_bytes bytes each
 * (two ping-pong field buffers and the Runge-Kutta residual), each 16-byte
 * aligned (the kernels copy rows with 16-byte loads; WDG_EINVAL otherwise).
 * They must stay valid until they are rebound or the context is destroyed. */
int32_t wdg_bind_state(wdg_ctx* ctx, void* q0, void* q1, void* res, int64_t bytes_each);

/* Copies fields in the canonical layout to / from the device (synchronous).
 * set_fields resets the residual, the step counter and the probe rows; it
 * keeps the time. */
int32_t wdg_set_fields(wdg_ctx* ctx, const double* q);
int32_t wdg_get_fields(wdg_ctx* ctx, double* q);
/* The Runge-Kutta residual buffer in the canonical layout (after wdg_rhs it
 * holds the right-hand side). */
int32_t wdg_get_residual(wdg_ctx* ctx, double* r);

int32_t wdg_set_time(wdg_ctx* ctx, double t);

/* Sets (or, with NULL, removes) the dipole source. */
int32_t wdg_set_dipole(wdg_ctx* ctx, const wdg_dipole* src);

/* Probe points xyz double [n][3]; each step appends one row of n x 6 values
 * (Ex..Hz) to a device buffer of `capacity` rows.  n = 0 removes probes. */
int32_t wdg_set_probes(wdg_ctx* ctx, int32_t n, const double* xyz, int32_t capacity);

/* Copies up to max_rows probe rows (double [rows][n][6]) to out and clears the
 * buffer (synchronous). */
int32_t wdg_probe_read(wdg_ctx* ctx, double* out, int32_t max_rows, int32_t* nrows);

/* Stage-kernel variants.  Both compute the same stage; they differ in how
 * the small dense products are executed.
 *   WDG_KERNEL_SCALAR: one wavefront per field component and 64 elements,
 *     reference operators as scalar FMA operands (any order and rule size);
 *   WDG_KERNEL_MFMA: six wavefronts (one per field component) per tile of 16
 *     elements, one or two tiles per workgroup, products on the matrix cores
 *     (the order / cubature sizes listed at wdg_set_kernel).
 * wdg_create selects MFMA when it is available. */
#define WDG_KERNEL_AUTO 0
#define WDG_KERNEL_SCALAR 1
#define WDG_KERNEL_MFMA 2

/* Selects the stage-kernel variant; WDG_EINVAL if MFMA is not available for
 * this order and cubature size (N=1,2: N_q <= 32; N=3: 17..48; N=4: 33..64)
 * or the E,H part of the state is 4 GiB or more (its lanes address neighbour
 * traces by 32-bit byte offsets: FP64 up to about 4.47M tetrahedra at N = 3,
 * 2.56M at N = 4, FP32 twice that); WDG_KERNEL_AUTO then takes SCALAR. */
int32_t wdg_set_kernel(wdg_ctx* ctx, int32_t variant);

/* ---- PML schemes compared with the weight-adjusted one ------------------- */

/* How the PML terms of eqs. (10)-(13) are evaluated.
 *   WDG_PML_WAA (default): the weight-adjusted scheme of eqs. (26)-(29), sigma
 *     (and kappa) at the cubature points, reference operators only.
 *   WDG_PML_DIRECT: the direct scheme with exact weighted mass matrices (the
 *     smoothly-varying implementation the paper compares against in Sec. I,
 *     the memory count after eq. (29) and Table I, "SV-paved"): for every PML
 *     element and axis u the library integrates the five mass matrices of
 *     eq. (15) weighted by a, b, c, d, 1/kappa of eq. (9), evaluated from the
 *     method's profile at the points of the rule passed here, and stores the
 *     products (M^a)^-1 M_k, (M^a)^-1 M^b, (M^a)^-1 M^c, M_k^-1 M^{1/kappa},
 *     M_k^-1 M^d: 15 N_p^2 words per PML element in the state's precision, read
 *     by every stage.
 *   WDG_PML_CONSTANT: element-constant coefficients (Sec. III, configuration
 *     (i), "EC-paved"): sigma_u and kappa_u of each PML element taken at its
 *     node farthest beyond the interface along +-u; the weighted mass matrices
 *     are then multiples of M_k and the PML terms are pointwise.
 * Elements carry auxiliary fields on the same set in every scheme (a nonzero
 * sigma or kappa != 1 at a cubature point).  Every scheme runs on the selected
 * stage kernel (wdg_set_kernel); the direct scheme adds a second launch per
 * stage that applies the stored products to the PML blocks and updates them. */
#define WDG_PML_WAA 0
#define WDG_PML_DIRECT 1
#define WDG_PML_CONSTANT 2

/* Selects the PML scheme.  For WDG_PML_DIRECT, nr points rst [nr][3] on the
 * reference tetrahedron (vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1))
 * with weights w [nr] integrate the weighted mass matrices (the weights are not
 * polynomial inside elements cut by the interface, so a rule well above degree
 * 2N is advisable); the other schemes ignore nr, rst and w.  Host setup in FP64
 * on up to 16 threads, then an upload; the previous scheme's data are freed.
 * Errors: WDG_EINVAL for an unknown scheme or a bad rule, WDG_ESTATE for a
 * host-only context or when sigma at the cubature points was replaced
 * (wdg_set_sigma_q, wdg_set_sigma_profile): these schemes sample the method's
 * profile, WDG_ENOMEM when the matrices do not fit. */
int32_t wdg_set_pml_scheme(wdg_ctx* ctx, int32_t scheme, int32_t nr, const double* rst, const double* w);

/* Tiles of 16 elements per workgroup of the matrix-core kernel: 1 or 2 (the
 * default where two fit in a compute unit's LDS; FP64 at N = 4 takes one,
 * WDG_EINVAL for two).  The per-element arithmetic is the same; the results
 * agree to rounding (the two are separately compiled kernels). */
int32_t wdg_set_tiles(wdg_ctx* ctx, int32_t tiles);

/* Times the available stage kernels (scalar-operand; matrix-core with 1 and 2
 * tiles per workgroup) over `reps` stage launches each on the current state
 * (best of three) and selects the fastest.  times_us double [3] (may be NULL)
 * receives the microseconds per launch, -1 where unavailable.  The fields are
 * unchanged; the Runge-Kutta residual is overwritten (a step starts by
 * resetting it).  Synchronises hip_stream. */
int32_t wdg_autotune(wdg_ctx* ctx, int32_t reps, double* times_us, void* hip_stream);

/* Like wdg_autotune, through a cache of chosen variants keyed by device
 * architecture, order, rule size, precision, PML scheme, kappa and the mesh's
 * size class (blocks rounded up to a power of two): a cached choice is applied
 * without timing (*from_cache = 1, may be NULL), otherwise the variants are
 * timed over `reps` launches and the choice is stored (*from_cache = 0).  The
 * cache lives in the process; when the environment variable
 * WDG_AUTOTUNE_CACHE names a file, entries are also read from it and appended
 * to it.  At creation the environment variables WDG_KERNEL (scalar | mfma)
 * and WDG_TILES (1 | 2) override the default variant (WDG_EINVAL from
 * wdg_create for other values or an unavailable choice). */
int32_t wdg_autotune_cached(wdg_ctx* ctx, int32_t reps, void* hip_stream, int32_t* from_cache);

/* Advances nsteps steps like wdg_step by replaying a captured HIP graph of two
 * steps (ten stage launches), re-captured when dt, the kernel choice or the
 * bound buffers change; an odd last step is launched directly.  Needs a
 * non-NULL stream, no dipole source and no probes (WDG_EINVAL): the source
 * amplitude and the probe row change every step. */
int32_t wdg_step_graph(wdg_ctx* ctx, double dt, int32_t nsteps, void* hip_stream);

#define WDG_SCHEDULE_FORWARD 0
#define WDG_SCHEDULE_REVERSED 1
#define WDG_SCHEDULE_ALTERNATING 2 /* the default */
/* Order in which workgroups take the element tiles (blocks) of a stage launch:
 * WDG_SCHEDULE_FORWARD (natural order), WDG_SCHEDULE_REVERSED, or
 * WDG_SCHEDULE_ALTERNATING (the default: successive stage launches alternate
 * between the two, so that a stage starts on the rows the previous one wrote
 * last, which are the ones still in the last-level cache when the state is
 * somewhat larger than it).  Every element's stage arithmetic reads only q_in
 * and writes only its own rows of q_out and the residual (ping-pong buffers),
 * so the results are bitwise identical in every order: a check for
 * cross-element read-after-write hazards.  WDG_EINVAL for another mode. */
int32_t wdg_set_schedule(wdg_ctx* ctx, int32_t mode);

/* The weight-adjusted inverse P_q a^-1 V_q of eq. (21) is applied to every PML
 * element's right-hand side by default, also where it is the identity: with
 * kappa = 1 the weight a of eq. (9) is one, and P_q V_q = I for a rule exact to
 * degree 2N.  on = 1 skips it there (a shortcut, exact to rounding; reported
 * separately from the default stage); on = 0 restores the default.  WDG_EINVAL
 * for on = 1 when the product is not the identity (kappa != 1, or
 * max |P_q V_q - I| >= 1e-12 for the context's rule). */
int32_t wdg_set_waa_shortcut(wdg_ctx* ctx, int32_t on);

/* Groups of independent simulations for captured stepping (contexts created
 * with WDG_ALIGN_COMPONENTS): group[k] (int32 [K], user element order) names
 * the group 0..ngroups-1 of element k; every face-connected component must lie
 * in one group, and each group must be a run of consecutive components
 * (components are numbered by their lowest element index).  wdg_step_graph
 * then captures, group after group, both steps of the pair for that group's
 * element blocks only, so that a group's fields stay in the last-level cache
 * over its ten stages; the arithmetic of every element is unchanged (results
 * bitwise equal to ungrouped stepping).  ngroups = 0 or group = NULL removes
 * the groups.  WDG_ESTATE for a context without aligned components, WDG_EINVAL
 * for groups that split a component or are not runs of consecutive
 * components. */
int32_t wdg_set_step_groups(wdg_ctx* ctx, int32_t ngroups, const int32_t* group);

/* Per-element factor on the time step, double [K] in user element order (NULL
 * removes it): element k advances with dt * scale[k], so independent
 * simulations held in one context (disjoint meshes) each keep their own stable
 * step.  Values must be positive and finite.  The context time advances by dt;
 * the source amplitude follows it. */
int32_t wdg_set_dt_scale(wdg_ctx* ctx, const double* scale);

/* Per-group PML profiles: element k of group group[k] (int32 [K], 0..ngroups-1)
 * gets sigma_u = sigma_max[g][u] (d_u / L_u)^order[g] at its cubature points
 * (interface box and thickness as given at creation; elements outside the PML
 * stay zero), so independent simulations in one context keep their own
 * conductivity.  Needs kappa = 1.  sigma_max double [ngroups][3], order
 * double [ngroups]. */
int32_t wdg_set_sigma_profile(wdg_ctx* ctx, const int32_t* group, int32_t ngroups, const double* sigma_max,
                              const double* order);

/* Advances nsteps LSERK4 steps of size dt, enqueued on hip_stream (a
 * hipStream_t; NULL for the default stream), without synchronising.
 * Returns WDG_EPROBE if the probe buffer would overflow. */
int32_t wdg_step(wdg_ctx* ctx, double dt, int32_t nsteps, void* hip_stream);

/* Evaluates the right-hand side of eqs. (26)-(29) at time t into the residual
 * buffer (fields unchanged), enqueued on hip_stream. */
int32_t wdg_rhs(wdg_ctx* ctx, double t, void* hip_stream);

/* Discrete energy 1/2 sum_k J_k (E^T M E + H^T M H) of the current fields,
 * accumulated in FP64 (synchronises hip_stream).  WDG_ENONFINITE if not finite. */
int32_t wdg_energy(wdg_ctx* ctx, double* out, void* hip_stream);

/* Host-side setup readouts (valid also for WDG_HOST_ONLY contexts). */
/* Physical node coordinates double [K][Np][3], user element order. */
int32_t wdg_node_coords(const wdg_ctx* ctx, double* xyz);

#define WDG_OP_DR 0   /* [Np][Np]   d l_j / dr at node i            */
#define WDG_OP_DS 1   /* [Np][Np]                                   */
#define WDG_OP_DT 2   /* [Np][Np]                                   */
#define WDG_OP_LIFT 3 /* [Np][4 Nfp] M^{-1} times face mass, eq. (17) */
#define WDG_OP_VQ 4   /* [Nq][Np]   V_q = V_I V^{-1}, eq. (20)      */
#define WDG_OP_PQ 5   /* [Np][Nq]   P_q = M^{-1} V_q^T W, eq. (21)  */
#define WDG_OP_M 6    /* [Np][Np]   reference mass matrix, eq. (14) */
/* FP64 reference operator `which` (row-major). */
int32_t wdg_reference_op(const wdg_ctx* ctx, int32_t which, double* out);

/* Per-element setup data in user element order; any pointer may be NULL.
 * J [K]; Fscale [K][4]; normals [K][4][3]; neighbour element and face
 * [K][4] (self for a wall); is_pml [K]. */
int32_t wdg_element_info(const wdg_ctx* ctx, double* J, double* Fscale, double* normals,
                         int32_t* etoe, int32_t* etof, int32_t* is_pml);

int32_t wdg_memory_report(const wdg_ctx* ctx, wdg_mem_t* out);

/* Device slot (block * 64 + lane of the blocked layout) of every element,
 * int32 [K] in user element order. */
int32_t wdg_element_slots(const wdg_ctx* ctx, int32_t* slot);

/* ---- Conductivity at the cubature points and differentiation ------------- */

/* sigma_u at the cubature points of every element (eqs. (9), (19)-(21): the PML
 * enters the scheme only through these samples), double [K][nq][3] in user
 * element order.  get returns the current values (zero outside the PML).  set
 * replaces them: values must be finite and zero on elements outside the PML
 * (they carry no auxiliary fields); WDG_EINVAL otherwise.  kappa is unchanged.
 * The arrays are copied. */
int32_t wdg_set_sigma_q(wdg_ctx* ctx, const double* sigma);
int32_t wdg_get_sigma_q(const wdg_ctx* ctx, double* sigma);

/* Physical cubature points double [K][nq][3], user element order. */
int32_t wdg_cubature_points(const wdg_ctx* ctx, double* xyz);

/* Re-samples sigma at the cubature points from the layer profile of Sec. III,
 * sigma_u = sigma_max[u] (d_u / L[u])^order, d_u the distance into the layer,
 * with new parameters (double [3], double [3], double).  The outer wall stays
 * where creation put it (interface +- thickness) and the interface moves with
 * L; the values then count as the method's profile again (grad_profile of
 * wdg_loss_gradient refers to these parameters).  Needs kappa = 1 and the
 * weight-adjusted scheme (WDG_ESTATE otherwise); WDG_EINVAL for L <= 0,
 * sigma_max < 0, order < 0, non-finite values, or a layer that would reach
 * elements created outside it (they carry no auxiliary fields). */
int32_t wdg_set_pml_profile(wdg_ctx* ctx, const double* sigma_max, const double* L, double order);

/* Axis-aligned shell: the points of the closed box [outer_lo, outer_hi] that
 * are not in the open box (inner_lo, inner_hi). */
typedef struct wdg_shell {
    double outer_lo[3], outer_hi[3];
    double inner_lo[3], inner_hi[3];
} wdg_shell;

/* Shell energy of the current fields in cubature form,
 * 1/2 sum_k J_k sum_q w_q chi(x_kq) (|E|^2 + |H|^2) at the cubature points
 * (fields interpolated with V_q, eq. (20)), accumulated in FP64.  Synchronises
 * hip_stream.  WDG_ENONFINITE if not finite. */
int32_t wdg_shell_energy(wdg_ctx* ctx, const wdg_shell* shell, double* out, void* hip_stream);

/* Loss J = sum_{n=1..nsteps} dt * shell_energy(q_n) over nsteps LSERK4 steps of
 * size dt from the current state, and its gradient from the discrete adjoint
 * of the scheme (energy inner product; the vacuum operator's adjoint is the
 * operator with the flux parameter negated, the PML terms of eqs. (26)-(29)
 * are transposed):
 *   grad_sigma   double [K][nq][3]: dJ/dsigma at the cubature points, zero
 *                outside the PML (NULL: not returned);
 *   grad_profile double [7]: dJ/d(sigma_max x,y,z, L x,y,z, profile order) of
 *                the profile given at creation or by wdg_set_pml_profile, with
 *                the outer wall fixed and the interface moving with L (NULL:
 *                not returned; WDG_ESTATE when sigma was replaced by
 *                wdg_set_sigma_q or wdg_set_sigma_profile, which no profile
 *                parameters describe).
 * The state advances by nsteps steps exactly as with wdg_step (no probe rows).
 * Forward states are checkpointed every checkpoint_interval steps (0:
 * ceil(sqrt(nsteps))) and every segment but the last is recomputed once during
 * the reverse sweep (the forward sweep keeps the last segment's stage inputs);
 * device memory for ceil(nsteps / interval) + 5 interval + 5 state buffers is
 * allocated and freed inside the call (a larger interval trades memory for
 * less recomputation: interval = nsteps recomputes nothing).  Needs kappa = 1
 * and an order and rule with a matrix-core kernel (WDG_EINVAL otherwise: FP64
 * at N = 4, N = 3 with more than 32 cubature points in FP64).  Synchronous. */
int32_t wdg_loss_gradient(wdg_ctx* ctx, double dt, int32_t nsteps, const wdg_shell* shell,
                          int32_t checkpoint_interval, double* loss, double* grad_sigma,
                          double* grad_profile, void* hip_stream);

/* ---- Allocation-free readout ---------------------------------------------- */

/* Largest mesh (in blocks of 64 element slots, per class) of wdg_energy_noalloc:
 * 32,768 blocks, a 256 KiB device array held by each GPU the library runs on. */
#define WDG_NOALLOC_MAX_BLOCKS 32768

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the energy
 * of wdg_energy, 1/2 sum_k J_k (E^T M E + H^T M H) of the current fields in
 * FP64, written to out_device (a device pointer to one double) on hip_stream,
 * without synchronising and without any allocation: the per-block partial sums
 * go to a fixed device array (WDG_NOALLOC_MAX_BLOCKS doubles) instead of the
 * context's scratch buffer.  The result is bitwise equal to wdg_energy's.
 * Calls on one GPU share that array: calls that overlap in time on one GPU
 * (two streams, two threads) race and must be ordered by the caller.  No
 * finiteness check (the value stays on the device).  WDG_EINVAL for a null
 * argument or a mesh of more than WDG_NOALLOC_MAX_BLOCKS blocks, WDG_ESTATE
 * for a host-only context or unbound state, WDG_EHIP on a launch error. */
int32_t wdg_energy_noalloc(wdg_ctx* ctx, double* out_device, void* hip_stream);

/* ---- Measurement helper --------------------------------------------------- */

/* Sustained rate of the matrix-core instructions the stage kernel uses for its
 * small dense products, measured on the current device: per 16x16x4 step one
 * V_MFMA_F32_16X16X4_F32 (FP32) or four V_MFMA_F64_4X4X4_4B_F64 (FP64), eight
 * workgroups of four wavefronts per compute unit, each wavefront running eight
 * independent accumulator chains of `iters` steps; best of three timed
 * launches after one untimed launch.  The roofline's measured compute peak;
 * not part of the method.  precision WDG_FP64 or WDG_FP32; *tflops receives
 * TFLOP/s (one multiply-add = 2 flops).  Allocates and frees a small device
 * buffer; synchronises hip_stream.  WDG_EINVAL for bad arguments, WDG_EHIP on
 * a launch error. */
int32_t wdg_measure_mfma_peak(int32_t precision, int32_t iters, void* hip_stream, double* tflops);

/* Device-memory bandwidth of a plain copy of `bytes` bytes (a multiple of 16,
 * at least 1 MiB) between two buffers allocated and freed inside the call:
 * 16-byte loads and stores, four per thread; best of five timed launches after
 * one untimed launch.  *gbs receives (bytes read + bytes written) / time in
 * GB/s.  Synchronises hip_stream.  WDG_EINVAL for bad arguments, WDG_ENOMEM,
 * WDG_EHIP on a launch error. */
int32_t wdg_measure_copy_bandwidth(int64_t bytes, void* hip_stream, double* gbs);

#ifdef __cplusplus
}
#endif

#endif /* WDG_H */
