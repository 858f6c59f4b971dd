/*
 * Plain FP64 CPU loops of the oracle (test infrastructure only).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU library.
 *
 * Contents:
 *   - element-scatter Galerkin assembly of the 2D stiffness matrix on a mapped
 *     geometry (Section 2, eq. (2); geometry of Section 4.3, quarter annulus as a
 *     B-spline surface) and of the load vector;
 *   - Gauss-Seidel smoothing on a CSR matrix, lexicographic and multicolour
 *     (smoothers of Algorithm 2; the paper notes Jacobi and Gauss-Seidel behave
 *     alike, Section 2.4);
 *   - CSR matrix-vector residual.
 *
 * Stencil storage used by the assembly: row I of the n x n interior grid
 * (I = i + n j, x index fastest) holds S = (2p+1)^2 entries, entry
 * o = (di + p) + (2p+1)(dj + p) being A[I, I + di + n dj].
 */
#include <math.h>
#include <stddef.h>
#include <string.h>

#define GEOM_IDENTITY 0
#define GEOM_ANNULUS 1

/* Quarter annulus with radii 1 and 2 written in closed form:
 * F(xi, eta) = (1 + xi) (1 - eta^2, 2 eta - eta^2).
 * Returns x, y and the Jacobian J = dF/d(xi, eta) (row-major, rows x/y). */
static void geometry_eval(int geom, double xi, double eta, double* X, double* Y,
                          double J[4]) {
    if (geom == GEOM_IDENTITY) {
        *X = xi;
        *Y = eta;
        J[0] = 1.0; J[1] = 0.0; J[2] = 0.0; J[3] = 1.0;
        return;
    }
    double r = 1.0 + xi;
    double cx = 1.0 - eta * eta;
    double cy = 2.0 * eta - eta * eta;
    *X = r * cx;
    *Y = r * cy;
    J[0] = cx;                   /* dx/dxi  */
    J[1] = r * (-2.0 * eta);     /* dx/deta */
    J[2] = cy;                   /* dy/dxi  */
    J[3] = r * (2.0 - 2.0 * eta);/* dy/deta */
}

/*
 * Element-scatter assembly of A_IJ = int grad(phi_I) . grad(phi_J) dx over the
 * mapped domain: on the reference square the integrand is
 * ghat_I^T D ghat_J with D = |det J| (J^T J)^{-1}.
 *
 * ne      elements per direction; p degree; nq Gauss points per direction
 * xq, wq  (ne*nq) physical Gauss points / weights of each 1D element
 * V, Dv   (ne*nq*(p+1)) values / derivatives of the p+1 functions alive on
 *         element e at its Gauss points (function e+a, a = 0..p)
 * first   1: drop the two Dirichlet functions per direction (n = ne + p - 2);
 *         0: keep every function (n = ne + p)
 * out     (n*n*S) stencil rows, zeroed here.
 * Elements are processed in (p+1) groups of rows ey so that no two elements
 * running in parallel touch the same matrix row.
 */
void orc_assemble_stiffness_2d(int ne, int p, int nq, int geom, int first,
                               const double* xq, const double* wq, const double* V,
                               const double* Dv, double* out) {
    const int n = ne + p - 2 * first;
    const int W = 2 * p + 1;
    const int S = W * W;
    const int P1 = p + 1;
    memset(out, 0, sizeof(double) * (size_t)n * n * S);
    for (int colour = 0; colour < P1; ++colour) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int ey = colour; ey < ne; ey += P1) {
            double gx[64], gy[64];
            for (int ex = 0; ex < ne; ++ex) {
                for (int qy = 0; qy < nq; ++qy) {
                    for (int qx = 0; qx < nq; ++qx) {
                        double X, Y, J[4];
                        double xi = xq[ex * nq + qx], eta = xq[ey * nq + qy];
                        geometry_eval(geom, xi, eta, &X, &Y, J);
                        double det = J[0] * J[3] - J[1] * J[2];
                        /* (J^T J) = [[a, b], [b, c]] */
                        double a = J[0] * J[0] + J[2] * J[2];
                        double b = J[0] * J[1] + J[2] * J[3];
                        double c = J[1] * J[1] + J[3] * J[3];
                        double idet = 1.0 / (a * c - b * b);
                        double w = wq[ex * nq + qx] * wq[ey * nq + qy] * fabs(det);
                        double D11 = w * c * idet, D12 = -w * b * idet, D22 = w * a * idet;
                        for (int a2 = 0; a2 < P1; ++a2)
                            for (int a1 = 0; a1 < P1; ++a1) {
                                int k = a1 + P1 * a2;
                                size_t ix = ((size_t)ex * nq + qx) * P1 + a1;
                                size_t iy = ((size_t)ey * nq + qy) * P1 + a2;
                                gx[k] = Dv[ix] * V[iy];
                                gy[k] = V[ix] * Dv[iy];
                            }
                        for (int a2 = 0; a2 < P1; ++a2) {
                            int jr = ey + a2 - first;
                            if (jr < 0 || jr >= n) continue;
                            for (int a1 = 0; a1 < P1; ++a1) {
                                int ir = ex + a1 - first;
                                if (ir < 0 || ir >= n) continue;
                                int ka = a1 + P1 * a2;
                                double* row = out + ((size_t)ir + (size_t)n * jr) * S;
                                for (int b2 = 0; b2 < P1; ++b2) {
                                    int jc = ey + b2 - first;
                                    if (jc < 0 || jc >= n) continue;
                                    for (int b1 = 0; b1 < P1; ++b1) {
                                        int ic = ex + b1 - first;
                                        if (ic < 0 || ic >= n) continue;
                                        int kb = b1 + P1 * b2;
                                        int o = (b1 - a1 + p) + W * (b2 - a2 + p);
                                        row[o] += D11 * gx[ka] * gx[kb] +
                                                  D12 * (gx[ka] * gy[kb] + gy[ka] * gx[kb]) +
                                                  D22 * gy[ka] * gy[kb];
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
    }
}

/*
 * Load vector b_I = int f phi_I dx on the mapped domain, with
 * f(x, y) = sum_m a_m sin(pi (k_m x + l_m y) + phi_m) evaluated at physical
 * points; modes holds (a, k, l, phi) per mode.  first = 1 drops the two
 * Dirichlet functions per direction (n = ne + p - 2), first = 0 keeps every
 * function (n = ne + p).
 */
void orc_assemble_load_2d(int ne, int p, int nq, int geom, int first, const double* xq,
                          const double* wq, const double* V, const double* modes,
                          int n_modes, double* out) {
    const int n = ne + p - 2 * first;
    const int P1 = p + 1;
    memset(out, 0, sizeof(double) * (size_t)n * n);
    for (int colour = 0; colour < P1; ++colour) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int ey = colour; ey < ne; ey += P1) {
            for (int ex = 0; ex < ne; ++ex)
                for (int qy = 0; qy < nq; ++qy)
                    for (int qx = 0; qx < nq; ++qx) {
                        double X, Y, J[4];
                        geometry_eval(geom, xq[ex * nq + qx], xq[ey * nq + qy], &X, &Y, J);
                        double det = J[0] * J[3] - J[1] * J[2];
                        double f = 0.0;
                        for (int m = 0; m < n_modes; ++m) {
                            const double* md = modes + 4 * m;
                            f += md[0] * sin(M_PI * (md[1] * X + md[2] * Y) + md[3]);
                        }
                        double w = wq[ex * nq + qx] * wq[ey * nq + qy] * fabs(det) * f;
                        for (int a2 = 0; a2 < P1; ++a2) {
                            int jr = ey + a2 - first;
                            if (jr < 0 || jr >= n) continue;
                            double vy = V[((size_t)ey * nq + qy) * P1 + a2];
                            for (int a1 = 0; a1 < P1; ++a1) {
                                int ir = ex + a1 - first;
                                if (ir < 0 || ir >= n) continue;
                                double vx = V[((size_t)ex * nq + qx) * P1 + a1];
                                out[(size_t)ir + (size_t)n * jr] += w * vx * vy;
                            }
                        }
                    }
        }
    }
}

/* Gauss-Seidel in natural (lexicographic) order: for I = 0..N-1, using the
 * newest values, x_I <- x_I + (b_I - (A x)_I) / A_II. */
void orc_gs_lex(int N, const int* indptr, const int* indices, const double* data,
                const double* diag, const double* b, double* x) {
    for (int I = 0; I < N; ++I) {
        double s = 0.0;
        for (int k = indptr[I]; k < indptr[I + 1]; ++k) s += data[k] * x[indices[k]];
        x[I] += (b[I] - s) / diag[I];
    }
}

/* Same sweep in reverse order (I = N-1..0): the backward half of a symmetric
 * Gauss-Seidel step. */
void orc_gs_lex_backward(int N, const int* indptr, const int* indices, const double* data,
                         const double* diag, const double* b, double* x) {
    for (int I = N - 1; I >= 0; --I) {
        double s = 0.0;
        for (int k = indptr[I]; k < indptr[I + 1]; ++k) s += data[k] * x[indices[k]];
        x[I] += (b[I] - s) / diag[I];
    }
}

/* One colour of multicolour Gauss-Seidel: every row listed in `rows` is updated
 * from the values x had at the start of this colour (two phases: all new values
 * are computed into tmp, then written back). */
void orc_gs_colour(int n_rows, const int* rows, const int* indptr, const int* indices,
                   const double* data, const double* diag, const double* b, double* x,
                   double* tmp) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n_rows; ++k) {
        int I = rows[k];
        double s = 0.0;
        for (int e = indptr[I]; e < indptr[I + 1]; ++e) s += data[e] * x[indices[e]];
        tmp[k] = x[I] + (b[I] - s) / diag[I];
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n_rows; ++k) x[rows[k]] = tmp[k];
}

/* r = b - A x for a CSR matrix. */
void orc_residual(int N, const int* indptr, const int* indices, const double* data,
                  const double* b, const double* x, double* r) {
#pragma omp parallel for schedule(static)
    for (int I = 0; I < N; ++I) {
        double s = 0.0;
        for (int k = indptr[I]; k < indptr[I + 1]; ++k) s += data[k] * x[indices[k]];
        r[I] = b[I] - s;
    }
}
