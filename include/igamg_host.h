/*
 * igamg_host.h -- host-only entry points of libigamg.so that expose the setup
 * arithmetic (no device work, usable without a GPU).  They return the same
 * tables the setup phase uploads, so that they can be checked on a CPU.
 *
 * Paper: Section 2.3 (open knot vectors, B-spline evaluation, Proposition 3)
 * and Section 2 (prolongation between nested spaces, Galerkin products).
 * All outputs are caller-owned host arrays of the documented size.
 */
#ifndef IGAMG_HOST_H
#define IGAMG_HOST_H

#ifdef __cplusplus
extern "C" {
#endif

/* Gauss-Legendre rule with m points on [-1, 1]: x[m], w[m].  Returns 0, or -1
 * for m < 1. */
int igamg_host_gauss_legendre(int m, double* x, double* w);

/* Values N[p+1] and derivatives dN[p+1] at u in [0, 1] of the p+1 B-splines of
 * the open uniform space (ne elements, degree p) that are alive on the element
 * containing u; *first receives the index of the first of them (0-based, all
 * functions counted).  Returns 0, or -1 for bad arguments. */
int igamg_host_basis(int ne, int p, double u, double* N, double* dN, int* first);

/* Dense 1D prolongation from ne_coarse to 2*ne_coarse elements computed by
 * knot insertion, all functions included: out[(2 ne_coarse + p) x (ne_coarse + p)]
 * row-major.  Returns 0, or -1 for bad arguments. */
int igamg_host_prolongation_1d(int ne_coarse, int p, double* out);

/* Interior 1D stiffness and mass bands (n = ne + p - 2 rows, 2p+1 columns,
 * column d+p holding A[i, i+d]) of level `level` of a hierarchy whose finest
 * grid has ne elements and whose coarsest has ne_coarsest (Galerkin products
 * below the finest level).  Returns 0, or -1 for bad arguments. */
int igamg_host_bands(int ne, int ne_coarsest, int level, int p, double* K, double* M);

/* Dense inverse inv[n x n] (row-major) of the coarsest-level operator A[n x n]
 * for Algorithm 2's direct coarsest solve, exactly as the setup phase forms
 * it: from the Cholesky factor A = L L^T when symmetric != 0 (the Poisson
 * operators, Section 2: A is SPD), else by Gauss-Jordan elimination with
 * partial pivoting (the nonsymmetric operators of Section 4.3).  Returns 0;
 * -4 (IGAMG_ENOTSPD) when a Cholesky pivot is not positive or an LU pivot
 * is below 1e-14 max|A| (inv untouched); -1 for bad arguments. */
int igamg_host_coarse_inverse(int n, const double* A, int symmetric, double* inv);

#ifdef __cplusplus
}
#endif

#endif /* IGAMG_HOST_H */
