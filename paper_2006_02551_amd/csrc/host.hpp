// Host-side setup of the WAA SC-PML DGTD library (FP64, C++17).
//
// Reference element (Sec. II-A, eqs. (14)-(21)), affine geometry and face
// connectivity (text after eq. (17)), PML sampling at cubature points
// (eqs. (19)-(20), Sec. II-B), element classification and the blocked device
// layout.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace wdg {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

using Mat = std::vector<double>;  // row-major dense matrix

// ---------------------------------------------------------------- refel.cpp
struct RefElement {
    int N = 0, Np = 0, Nfp = 0, Nq = 0;
    std::vector<double> r, s, t;         // nodes [Np]
    std::vector<int> fmask;              // [4][Nfp]
    Mat V, Vinv, M, Minv;                // [Np][Np]
    Mat Dr, Ds, Dt;                      // [Np][Np]
    Mat LIFT;                            // [Np][4 Nfp]
    Mat Vq;                              // [Nq][Np]
    Mat Pq;                              // [Np][Nq]
    std::vector<double> rq, sq, tq, wq;  // cubature [Nq]
};

// Builds every reference operator for order N and the given cubature rule.
RefElement build_reference(int N, int nq, const double* rst, const double* w);

// Orthonormal basis values at (r,s,t) for all Np modes.
void ortho_basis(int N, double r, double s, double t, double* out);

// Dense helpers.
Mat matmul(const Mat& A, const Mat& B, int n, int k, int m);
Mat invert(const Mat& A, int n);
Mat transpose(const Mat& A, int n, int m);

// ----------------------------------------------------------------- mesh.cpp
struct PmlParams {
    double lo[3], hi[3], L[3], sigma_max[3];
    double order, kappa_max;
};

// (d / L)^p with d the distance of x beyond [lo, hi] (0 inside; p = 0 gives a step).
double profile_ratio(double x, double lo, double hi, double L, double p);

struct Setup {
    RefElement ref;
    int K = 0, K_pml = 0;
    int B = 64;               // elements per block
    int nblk_pml = 0, nblk = 0;
    bool has_kappa = false;
    double flux_alpha = 1.0;
    // user order geometry
    std::vector<int> etov;               // [K][4], reoriented
    std::vector<double> vxyz;            // [nv][3]
    std::vector<double> J;               // [K]
    std::vector<double> metric;          // [K][9]  rx ry rz sx sy sz tx ty tz
    std::vector<double> nrm;             // [K][4][3]
    std::vector<double> Fscale;          // [K][4]
    std::vector<int> etoe, etof;         // [K][4]
    std::vector<int> nbr_node;           // [K][4][Nfp] neighbour volume node (or own node at walls)
    std::vector<double> xnodes;          // [K][Np][3]
    std::vector<double> sigma, kappa;    // [K][Nq][3]
    std::vector<double> xq;              // [K][Nq][3] physical cubature points
    PmlParams pml{};                     // the profile sigma and kappa were sampled from
    std::vector<int> is_pml;             // [K]
    // device ordering
    std::vector<int> perm;               // user element -> slot (blk*B + lane)
    std::vector<int> slot_elem;          // slot -> user element or -1
    // face-connected components (independent simulations of a batch), numbered by their lowest element
    int ncomp = 0;
    std::vector<int> comp;               // [K] component of each element
    // with aligned components: blocks [blk0, blk1) of each component in the PML class and in the vacuum
    // class (empty ranges otherwise)
    bool aligned = false;
    std::vector<int> comp_pml0, comp_pml1, comp_int0, comp_int1;
    double dt_unit = 0.0;
};

// vertex_id: null, or [nv] identification used by the face connectivity (periodic meshes).
// align_components: every face-connected component starts at a block boundary in each class.
Setup build_setup(int nv, const double* vxyz, int K, const int* etov, const int* vertex_id, int N, int nq,
                  const double* rst, const double* w, const PmlParams& pml, double flux_alpha,
                  bool align_components = false);

// Element containing a point (largest smallest barycentric coordinate, lowest
// index on ties) and the Lagrange weights [Np] at it.
int locate_point(const Setup& S, const double* x, double* weights);

}  // namespace wdg
