// One-dimensional model problem of Section 2.4 (eq. (6)): -u'' = (2 pi)^2 sin(2 pi x)
// on (0, 1) with homogeneous Dirichlet conditions, B-splines of degree 1..9.
//
// A 1D problem has at most a few thousand unknowns, far too few to fill the
// chip, so each problem of a set is solved by ONE workgroup in ONE launch:
// Algorithm 5 (restarted RRE/MPE, Algorithms 3 and 4) around mu-cycles of
// Algorithm 2, with every level's iterate, right-hand side and residual in LDS,
// the (2p+1)-wide bands too when they fit beside them (staged once per launch),
// and the transfer tables and coarsest inverse read through the caches.  The
// iterates s_0 .. s_{q+1} and the orthonormal columns of the QR factorisation
// live in a per-problem global workspace, touched once per cycle.  A set of problems occupies one workgroup per problem (one per CU).
#pragma once

namespace igamg {

constexpr int kMax1DLevels = 16;
constexpr int kMax1DDegree = 9;
constexpr int kLds1D = 16384;  // doubles of LDS: x, b, r of every level, then the bands if they fit (128 KB)

struct Desc1D {
    int p, L, n_el, nq;
    int smoother, nu1, nu2, mu, method, q;
    double omega;
    int n[kMax1DLevels];    // unknowns of level l
    int off[kMax1DLevels];  // LDS offset of x_l; b_l and r_l follow, n_l each
    int bands_lds;          // 1: every level's band is copied to LDS at boff[l]
    int boff[kMax1DLevels];
    const double* K[kMax1DLevels];  // n_l x (2p+1) bands: K[i*(2p+1) + d + p] = A_l[i, i+d]
    const int* rs[kMax1DLevels];    // restriction of level l (to l-1): windows and weights
    const double* rw[kMax1DLevels];
    int RW[kMax1DLevels];
    const int* ps[kMax1DLevels];    // prolongation of level l (from l-1)
    const double* pw[kMax1DLevels];
    int PW[kMax1DLevels];
    const double* Ainv0;  // n_0 x n_0 inverse of the coarsest matrix
    const double* b;      // finest right-hand side
    double* S;            // (q+2) x n_L iterates
    double* Qm;           // (q+1) x n_L orthonormal columns
    const double* V;      // basis values at the Gauss points: ((e*nq + g)*(p+1) + a)
    const double* wq;     // Gauss weights and points, e*nq + g
    const double* xq;
};

struct Out1D {
    int restarts, vcycles, breakdowns, converged, status;
    double rel_residual, l2_error;
};

// b_i = int f N_{i+1} by the element Gauss rule, elements in increasing order.
__global__ void k_load1d(int n_el, int p, int nq, const double* __restrict__ V, const double* __restrict__ wq,
                         const double* __restrict__ xq, double* __restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = n_el + p - 2;
    if (i >= n) return;
    const int k = i + 1;  // function index in the full basis 0 .. n_el + p - 1
    double acc = 0.0;
    for (int e = max(0, k - p); e <= min(n_el - 1, k); ++e) {
        const int a = k - e;
        for (int g = 0; g < nq; ++g) {
            const int t = e * nq + g;
            const double x = xq[t];
            const double f = (2.0 * M_PI) * (2.0 * M_PI) * sin(2.0 * M_PI * x);
            acc += wq[t] * f * V[(size_t)t * (p + 1) + a];
        }
    }
    b[i] = acc;
}

// Sum over the workgroup (kBlock threads); every thread gets the same value.
__device__ inline double block_sum1d(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();  // red may still be read by the previous call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    return s;
}

// The first cnt entries of h summed over the workgroup, in place.
__device__ inline void block_sum1d_vec(double* h, int cnt, double* red) {
#pragma unroll
    for (int k = 0; k < kMaxCols; ++k) {
        if (k < cnt) {
            double v = h[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            h[k] = v;
        }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < kMaxCols; ++k)
            if (k < cnt) red[(threadIdx.x >> 6) * kMaxCols + k] = h[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxCols; ++k) {
        if (k < cnt) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) s += red[w * kMaxCols + k];
            h[k] = s;
        }
    }
}

// (A_l x)_i over the columns of row i that exist.
__device__ inline double band_row(const double* __restrict__ K, const double* x, int i, int n, int p) {
    const int W = 2 * p + 1;
    const double* k = K + (size_t)i * W;
    const int lo = max(0, p - i), hi = min(W, n - i + p);
    double s = 0.0;
    for (int d = lo; d < hi; ++d) s = fma(k[d], x[i + d - p], s);
    return s;
}

struct Work1D {
    const Desc1D& D;
    double* lds;
    double* red;

    __device__ double* x(int l) const { return lds + D.off[l]; }
    __device__ const double* band(int l) const { return D.bands_lds ? lds + D.boff[l] : D.K[l]; }
    __device__ double* b(int l) const { return lds + D.off[l] + D.n[l]; }
    __device__ double* r(int l) const { return lds + D.off[l] + 2 * D.n[l]; }

    // nsweeps smoothing steps on level l: lexicographic Gauss-Seidel, weighted
    // Jacobi, or multicolour Gauss-Seidel with the p+1 colours i mod (p+1),
    // colours in increasing order (rows of one colour are more than p apart, so
    // they do not couple).
    __device__ void smooth(int l, int nsweeps) const {
        const int n = D.n[l], p = D.p, W = 2 * p + 1;
        const double* K = band(l);
        double *xl = x(l), *bl = b(l), *rl = r(l);
        for (int s = 0; s < nsweeps; ++s) {
            if (D.smoother == IGAMG_SMOOTH_LEXGS) {
                // forward sweep, i increasing: each row needs the new values of
                // the p rows before it, a strict recurrence run by one thread
                if (threadIdx.x == 0)
                    for (int i = 0; i < n; ++i)
                        xl[i] = xl[i] + (bl[i] - band_row(K, xl, i, n, p)) / K[(size_t)i * W + p];
                __syncthreads();
            } else if (D.smoother == IGAMG_SMOOTH_JACOBI) {
                for (int i = threadIdx.x; i < n; i += kBlock)
                    rl[i] = (bl[i] - band_row(K, xl, i, n, p)) / K[(size_t)i * W + p];
                __syncthreads();
                for (int i = threadIdx.x; i < n; i += kBlock) xl[i] += D.omega * rl[i];
                __syncthreads();
            } else {
                for (int c = 0; c <= p; ++c) {
                    for (int i = c + (p + 1) * threadIdx.x; i < n; i += (p + 1) * kBlock)
                        xl[i] = xl[i] + (bl[i] - band_row(K, xl, i, n, p)) / K[(size_t)i * W + p];
                    __syncthreads();
                }
            }
        }
    }

    // r_l = b_l - A_l x_l; b_{l-1} = P_l^T r_l; x_{l-1} = 0.
    __device__ void restrict_residual(int l) const {
        const int n = D.n[l], nc = D.n[l - 1], p = D.p, RW = D.RW[l];
        const double* K = band(l);
        double *xl = x(l), *bl = b(l), *rl = r(l);
        for (int i = threadIdx.x; i < n; i += kBlock) rl[i] = bl[i] - band_row(K, xl, i, n, p);
        __syncthreads();
        const int* rs = D.rs[l];
        const double* rw = D.rw[l];
        double *bc = b(l - 1), *xc = x(l - 1);
        for (int I = threadIdx.x; I < nc; I += kBlock) {
            const double* w = rw + (size_t)I * RW;
            const double* src = rl + rs[I];
            // on grids narrower than the window its zero-weight tail leaves the level
            const int m = min(RW, n - rs[I]);
            double s = 0.0;
            for (int a = 0; a < m; ++a) s = fma(w[a], src[a], s);
            bc[I] = s;
            xc[I] = 0.0;
        }
        __syncthreads();
    }

    // x_l += P_l x_{l-1}.
    __device__ void prolong(int l) const {
        const int n = D.n[l], nc = D.n[l - 1], PW = D.PW[l];
        const int* ps = D.ps[l];
        const double* pw = D.pw[l];
        double *xl = x(l), *xc = x(l - 1);
        for (int i = threadIdx.x; i < n; i += kBlock) {
            const double* w = pw + (size_t)i * PW;
            const double* src = xc + ps[i];
            const int m = min(PW, nc - ps[i]);
            double s = 0.0;
            for (int a = 0; a < m; ++a) s = fma(w[a], src[a], s);
            xl[i] += s;
        }
        __syncthreads();
    }

    // x_0 = A_0^{-1} b_0 (the initial guess does not enter).
    __device__ void coarse() const {
        const int n0 = D.n[0];
        double *x0 = x(0), *b0 = b(0);
        for (int i = threadIdx.x; i < n0; i += kBlock) {
            const double* a = D.Ainv0 + (size_t)i * n0;
            double s = 0.0;
            for (int j = 0; j < n0; ++j) s = fma(a[j], b0[j], s);
            x0[i] = s;
        }
        __syncthreads();
    }

    // One mu-cycle on the finest level (Algorithm 2) without recursion: each
    // level counts the coarse-grid visits it has made; a revisit smooths and
    // restricts again from the coarse iterate in place.
    __device__ void cycle() const {
        const int L = D.L;
        if (L == 0) {
            coarse();
            return;
        }
        int cnt[kMax1DLevels];
        int l = L;
        bool down = true;
        while (true) {
            if (down) {
                if (l == 0) {
                    coarse();
                    down = false;
                    l = 1;
                    continue;
                }
                smooth(l, D.nu1);
                restrict_residual(l);
                cnt[l] = 0;
                --l;
            } else {
                if (++cnt[l] < D.mu) {
                    --l;
                    down = true;
                    continue;
                }
                prolong(l);
                smooth(l, D.nu2);
                if (l == L) break;
                ++l;
            }
        }
    }

    // ||b_L - A_L x_L||_2 (uses r_L as scratch).
    __device__ double residual_norm() const {
        const int L = D.L, n = D.n[L], p = D.p;
        const double* K = band(L);
        const double *xl = x(L), *bl = b(L);
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += kBlock) {
            const double v = bl[i] - band_row(K, xl, i, n, p);
            s += v * v;
        }
        return sqrt(block_sum1d(s, red));
    }

    __device__ void store(double* dst) const {
        const int n = D.n[D.L];
        const double* xl = x(D.L);
        for (int i = threadIdx.x; i < n; i += kBlock) dst[i] = xl[i];
    }
};

// mode 0: solve to tol (max_iters restarts, or V-cycles for method 0);
// mode 1: apply max_iters cycles.  x_dev[blockIdx.x] holds the initial guess
// and receives the result.
__global__ void __launch_bounds__(kBlock) k_solve1d(const Desc1D* __restrict__ descs, double* const* __restrict__ xs,
                                                    int mode, int max_iters, double tol, Out1D* __restrict__ outs) {
    __shared__ double lds[kLds1D];
    __shared__ double red[(kBlock / 64) * kMaxCols];
    __shared__ double Rs[kMaxCols * kMaxCols];
    __shared__ ExtrapCoeffs cf;
    const Desc1D& D = descs[blockIdx.x];
    Work1D w{D, lds, red};
    const int L = D.L, n = D.n[L];
    double* xg = xs[blockIdx.x];
    {
        double *xl = w.x(L), *bl = w.b(L);
        for (int i = threadIdx.x; i < n; i += kBlock) {
            xl[i] = xg[i];
            bl[i] = D.b[i];
        }
        if (D.bands_lds) {
            const int W = 2 * D.p + 1;
            for (int l = 0; l <= L; ++l) {
                double* dst = lds + D.boff[l];
                const double* src = D.K[l];
                for (int e = threadIdx.x; e < D.n[l] * W; e += kBlock) dst[e] = src[e];
            }
        }
        __syncthreads();
    }
    Out1D o{0, 0, 0, 0, 0, 0.0, 0.0};
    double bsq = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) bsq += D.b[i] * D.b[i];
    // ||b|| (1 for a zero right-hand side, whose test is then absolute)
    const double bn = sqrt(block_sum1d(bsq, red)), bnorm = bn > 0.0 ? bn : 1.0;
    if (mode == 1) {
        for (int k = 0; k < max_iters; ++k) {
            w.cycle();
            ++o.vcycles;
        }
    } else if (D.method == 0) {
        for (int k = 0; k < max_iters; ++k) {
            w.cycle();
            ++o.vcycles;
            ++o.restarts;
            o.rel_residual = w.residual_norm() / bnorm;
            if (!isfinite(o.rel_residual)) {
                o.status = -7;
                break;
            }
            if (o.rel_residual <= tol) {
                o.converged = 1;
                break;
            }
        }
    } else {
        const int q = D.q, nc = q + 1;
        double* xl = w.x(L);
        double* v = w.r(L);
        for (int k = 0; k < max_iters; ++k) {
            // every copy of x_L completes before the next cycle rewrites it
            for (int i = threadIdx.x; i < n; i += kBlock) D.S[i] = xl[i];
            __syncthreads();
            for (int j = 1; j <= nc; ++j) {
                w.cycle();
                ++o.vcycles;
                double* sj = D.S + (size_t)j * n;
                for (int i = threadIdx.x; i < n; i += kBlock) sj[i] = xl[i];
                __syncthreads();
            }
            // QR of Delta S = [s_1 - s_0, ..., s_{q+1} - s_q] by Gram-Schmidt
            // applied twice (R equals Householder's R up to row signs)
            for (int j = 0; j < nc; ++j) {
                const double* s0 = D.S + (size_t)j * n;
                const double* s1 = s0 + n;
                for (int i = threadIdx.x; i < n; i += kBlock) v[i] = s1[i] - s0[i];
                double racc[kMaxCols];
#pragma unroll
                for (int kk = 0; kk < kMaxCols; ++kk) racc[kk] = 0.0;
                for (int pass = 0; pass < 2 && j > 0; ++pass) {
                    double h[kMaxCols];
#pragma unroll
                    for (int kk = 0; kk < kMaxCols; ++kk) h[kk] = 0.0;
                    __syncthreads();
                    for (int i = threadIdx.x; i < n; i += kBlock) {
                        const double vi = v[i];
#pragma unroll
                        for (int kk = 0; kk < kMaxCols; ++kk)
                            if (kk < j) h[kk] = fma(D.Qm[(size_t)kk * n + i], vi, h[kk]);
                    }
                    block_sum1d_vec(h, j, red);
                    for (int i = threadIdx.x; i < n; i += kBlock) {
                        double vi = v[i];
#pragma unroll
                        for (int kk = 0; kk < kMaxCols; ++kk)
                            if (kk < j) vi = fma(-h[kk], D.Qm[(size_t)kk * n + i], vi);
                        v[i] = vi;
                    }
#pragma unroll
                    for (int kk = 0; kk < kMaxCols; ++kk) racc[kk] += h[kk];
                }
                __syncthreads();
                double ss = 0.0;
                for (int i = threadIdx.x; i < n; i += kBlock) ss += v[i] * v[i];
                const double nrm = sqrt(block_sum1d(ss, red));
                if (threadIdx.x == 0) {
                    for (int kk = 0; kk < nc; ++kk)
                        Rs[kk * nc + j] = kk < j ? racc[kk] : (kk == j ? nrm : 0.0);
                }
                const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
                double* qj = D.Qm + (size_t)j * n;
                for (int i = threadIdx.x; i < n; i += kBlock) qj[i] = v[i] * inv;
                __syncthreads();
            }
            if (threadIdx.x == 0) cf = extrap_coefficients(Rs, nc, D.method);
            __syncthreads();
            const int info = cf.info;
            if (info == -2) {
                o.status = -7;
                break;
            }
            if (info == -1) {
                ++o.breakdowns;
                const double* sl = D.S + (size_t)nc * n;
                for (int i = threadIdx.x; i < n; i += kBlock) xl[i] = sl[i];
            } else {
                // t = s_0 + sum_{j<q} alpha_j (s_{j+1} - s_j)
                for (int i = threadIdx.x; i < n; i += kBlock) {
                    double t = D.S[i];
                    for (int j = 0; j < q; ++j)
                        t = fma(cf.alpha[j], D.S[(size_t)(j + 1) * n + i] - D.S[(size_t)j * n + i], t);
                    xl[i] = t;
                }
            }
            __syncthreads();
            ++o.restarts;
            o.rel_residual = w.residual_norm() / bnorm;
            if (!isfinite(o.rel_residual)) {
                o.status = -7;
                break;
            }
            if (o.rel_residual <= tol) {
                o.converged = 1;
                break;
            }
        }
    }
    __syncthreads();
    w.store(xg);
    // L2 error against u = sin(2 pi x) with the element Gauss rule
    {
        const int p = D.p, nq = D.nq, ne = D.n_el;
        const double* xl = w.x(L);
        double e2 = 0.0;
        for (int t = threadIdx.x; t < ne * nq; t += kBlock) {
            const int e = t / nq;
            const double* Vt = D.V + (size_t)t * (p + 1);
            double u = 0.0;
            for (int a = 0; a <= p; ++a) {
                const int kf = e + a;  // full-basis index; interior unknown kf - 1
                if (kf >= 1 && kf <= n) u = fma(Vt[a], xl[kf - 1], u);
            }
            const double d = u - sin(2.0 * M_PI * D.xq[t]);
            e2 += D.wq[t] * d * d;
        }
        o.l2_error = sqrt(block_sum1d(e2, red));
    }
    if (threadIdx.x == 0) outs[blockIdx.x] = o;
}

}  // namespace igamg
