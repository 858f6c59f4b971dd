// Host-side univariate B-spline machinery used by the setup phase.
//
// Paper: Section 2.3 (open uniform knot vectors, B-splines and their local
// support, Proposition 3) and Section 2 (nested coarse/fine spaces,
// prolongation P and Galerkin coarse operators, eq. (4)).
#pragma once

#include <cstddef>
#include <vector>

namespace igamg {

// Open uniform knots (0^{p+1}, 1/ne, ..., (ne-1)/ne, 1^{p+1}).
std::vector<double> open_knots(int ne, int p);

// Gauss-Legendre rule with m points on [-1, 1] (Newton on P_m).
void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w);

// Values and first derivatives of the p+1 B-splines alive on span
// [t_s, t_{s+1}) at u (de Boor's triangular scheme): N[r], dN[r] belong to
// function s - p + r.
void basis_and_derivs(const std::vector<double>& t, int p, int s, double u, double* N,
                      double* dN);

// Per-element tables for ne elements, nq Gauss points, degree p:
// pts/wts[e*nq + q] (physical), V/D[(e*nq + q)*(p+1) + a] for function e + a.
struct ElementTables {
    int ne, nq, p;
    std::vector<double> pts, wts, V, D;
};
ElementTables element_tables(int ne, int p, int nq);

// Values at arbitrary points x_k of the p+1 functions alive on the span that
// contains x_k in a grid of ne elements: out span index and tables.
void eval_at_points(int ne, int p, const std::vector<double>& x, std::vector<int>& span,
                    std::vector<double>& V, std::vector<double>& D);

// Sparse column representation of the 1D prolongation from nc to 2*nc elements
// computed by Boehm knot insertion of all midpoints.  col_start[J] is the first
// fine function with a nonzero in column J, col_val[J] the values.  All
// functions (Dirichlet ones included).
struct Prolong1D {
    int nc_el, nf_fun, nc_fun, p;
    std::vector<int> col_start;
    std::vector<std::vector<double>> col_val;
};
Prolong1D prolongation_boehm(int nc_el, int p);

// Interior (Dirichlet-free) transfer tables between n_c and n_f interior
// unknowns.  Restriction: coarse row I gathers fine entries
// r_start[I] .. r_start[I] + RW - 1 with weights r_w[I*RW + a] (zero padded,
// r_start clamped so that the window stays inside [0, n_f)).  Prolongation:
// fine row i gathers coarse entries p_start[i] .. + PW - 1 with p_w[i*PW + a].
struct TransferTables {
    int nf, nc, RW, PW;
    std::vector<int> r_start, p_start;
    std::vector<double> r_w, p_w;
};
TransferTables transfer_tables(const Prolong1D& P);

// Banded 1D matrices: band[i*(2p+1) + (d+p)] = A[i, i+d], zero outside.
struct Band1D {
    int n, p;
    std::vector<double> v;
    double at(int i, int d) const { return v[(size_t)i * (2 * p + 1) + d + p]; }
};
// Interior 1D stiffness and mass matrices by Gauss quadrature (p+1 points).
void stiffness_mass_bands(int ne, int p, Band1D& K, Band1D& M);
// Galerkin product P^T A P of a banded interior matrix on the fine level.
Band1D galerkin_band(const Band1D& Af, const TransferTables& T, int p);

// Dense SPD Cholesky A = L L^T (lower, in place, row-major n x n).  Returns
// false when a pivot is not positive.
bool cholesky_inplace(std::vector<double>& A, int n);
// A^{-1} from its Cholesky factor (row-major n x n).
std::vector<double> inverse_from_cholesky(const std::vector<double>& L, int n);
// Inverse of a dense row-major n x n matrix by Gauss-Jordan elimination with
// partial pivoting (nonsymmetric coarsest operators); false if singular.
bool inverse_lu(const std::vector<double>& A, int n, std::vector<double>& inv);
// Dense inverse of the coarsest operator (Algorithm 2's direct solve): from
// the Cholesky factor when `symmetric`, else by LU.  Returns 0, or -4 (the
// library's ENOTSPD) when a Cholesky pivot is not positive or the LU pivot
// vanishes; inv is then unchanged.
int coarse_inverse(std::vector<double> A, int n, bool symmetric, std::vector<double>& inv);

}  // namespace igamg
