// Host-side structures shared by the setup (setup.cpp) and the device engine
// (engine.hip).  Nothing here touches the GPU.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "amg_eig.h"

namespace amgeig {

struct Csr {
    int64_t nr = 0, nc = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

// One level of the hierarchy, k = 0 is the finest.
struct Level {
    int64_t n = 0;
    // A_k and M_k on one shared pattern (explicit zeros kept), FP64.
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> a, m;
    // The V-cycle operator A_k - sigma M_k without explicit off-diagonal zeros
    // (A_k itself without a shift), and its l1 diagonal.
    Csr av;
    std::vector<double> l1;   // d_i = sum_j |av_ij|
    std::vector<int32_t> cf;  // C/F splitting towards level k+1 (1 = C)
    Csr P, Pt;                // prolongation n_k x n_{k+1} and its transpose
    // Multicolour Gauss-Seidel (only with that smoother): first-fit colours of
    // the graph of av, the rows colour by colour (ascending within a colour),
    // the colour boundaries in that sequence, and av's rows in that sequence
    // without their diagonal: all off-diagonal entries (gs_all) and those
    // whose column has a smaller colour than the row (gs_lo), plus a_ii.
    std::vector<int32_t> colour, corder;
    std::vector<int64_t> coff;
    Csr gs_all, gs_lo;
    std::vector<double> gs_diag;
};

struct Hierarchy {
    std::vector<Level> lv;
    int dn = 0;
    std::vector<double> lam;   // coarsest eigenvalues, ascending
    std::vector<double> Z;     // dn x dn row-major, column j = eigenvector j, Z^T M_n Z = I
    std::vector<double> Ainv;  // dn x dn row-major, (A_n - sigma M_n)^-1 = Z diag(1/(lam - sigma)) Z^T
    double sigma = 0.0;        // shift of the V-cycle operators A_k - sigma M_k (0: none)
};

// Status codes of amg_eig.h, returned by the setup routines.
int build_hierarchy(const amg_eig_csr *A, const amg_eig_csr *M, int q, const amg_eig_opts &o, Hierarchy &H,
                    int &qe, std::string &err);

// Dense symmetric-definite eigen-decomposition (host, FP64): A z = lam M z with
// Z^T M Z = I, eigenvalues ascending.  A and M row-major n x n.  Returns false if
// M is not positive definite.
bool dense_sygv(int n, const std::vector<double> &A, const std::vector<double> &M, std::vector<double> &lam,
                std::vector<double> &Z);

// Coarsen on the device with PMIS (setup_device.hip): from H.lv.back() on,
// while H.lv.size() < max_levels and the last level has more than coarse_max
// rows, form strength, splitting, P, P^T and the next level on the current
// device and append it (cf, P, Pt of each coarsened level filled); a splitting
// with fewer than cmin or more than 0.9 n C points ends the loop.  Returns an
// amg_eig status code.
int device_coarsen(Hierarchy &H, const amg_eig_opts &o, int64_t cmin, std::string &err);

// dense_sygv on the current device (amg_eig_dense_sygv); returns a status code.
int device_sygv(int n, const std::vector<double> &A, const std::vector<double> &M, std::vector<double> &lam,
                std::vector<double> &Z, std::string &err);

// Choose the block width by the guard rule on approximate eigenvalues.
int guard_width(const std::vector<double> &lam, int q, double gap, int cap);

}  // namespace amgeig
