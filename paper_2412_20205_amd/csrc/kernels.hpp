// Device kernels of the extrapolated multigrid solver (gfx950, wave64).
//
// Operators (Section 2, eq. (2)):
//   Stencil2D  -- (2p+1)^2 stored FP64/FP32 coefficients per unknown, laid out
//                 colour-blocked: for colour c and its k-th point the entry of
//                 offset o sits at coef[(c*S + o)*ncp + k], so one colour pass
//                 streams S contiguous arrays (coalesced, read once).
//   Kron2D/3D  -- unit square/cube operators K(x)M + M(x)K (+ third term in 3D)
//                 applied from banded 1D factors, sum-factorised per row.
// Smoother: multicolour Gauss-Seidel, colour c(I) = sum_d (i_d mod (p+1))(p+1)^d,
// one launch per colour; x_I <- x_I + (b_I - (A x)_I) / A_II.
// Transfers: separable knot-insertion prolongation P = P1 (x) P1 (x) P1 and
// R = P^T from per-index 1D weight windows.
// Extrapolation (Algorithms 3 and 4): tall-skinny Householder QR tree of the
// difference matrix, one-thread small solve, streaming combination.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace igamg {

// ---------------------------------------------------------------------------
// helpers

// Workgroups are dealt round-robin to the XCDs.  Remap so that consecutive
// logical tiles run on the same XCD and share its L2 (neighbour rows of x).
__device__ __forceinline__ int xcd_swizzle(int bid, int nblk) {
    int q = nblk / kNumXcd, r = nblk % kNumXcd;
    int x = bid % kNumXcd, s = bid / kNumXcd;
    return (x < r) ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
    return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum (fixed tree order); result valid in every thread.
__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// ---------------------------------------------------------------------------
// operators

struct Pt2 {
    int i, j;
    long long I;
};
struct Pt3 {
    int i, j, k;
    long long I;
};

template <int P, typename T_>
struct Stencil2D {
    using T = T_;
    using Pt = Pt2;
    static constexpr int W = 2 * P + 1, S = W * W, NC = (P + 1) * (P + 1);
    static constexpr bool kColourOrder = true;
    const T* __restrict__ coef;
    int n;
    int ncp;

    __device__ __forceinline__ int colour_size(int c) const {
        int ci = c % (P + 1), cj = c / (P + 1);
        int ni = (n - ci + P) / (P + 1), nj = (n - cj + P) / (P + 1);
        return ni * nj;
    }
    __device__ __forceinline__ bool point(int c, int k, Pt& pt) const {
        int ci = c % (P + 1), cj = c / (P + 1);
        int ni = (n - ci + P) / (P + 1), nj = (n - cj + P) / (P + 1);
        if (k >= ni * nj) return false;
        int jj = k / ni, ii = k - jj * ni;
        pt.i = ci + (P + 1) * ii;
        pt.j = cj + (P + 1) * jj;
        pt.I = pt.i + (long long)n * pt.j;
        return true;
    }
    static constexpr int NW = W;  // one slice per stencil row
    // Partial row product over stencil row bb = w - P (coefficients streamed
    // once, coalesced across the 64 points of the wave); diag set by w == P.
    __device__ __forceinline__ T slice(const T* __restrict__ x, const Pt& pt, int c, int k, int w,
                                       T& diag) const {
        const int bb = w - P;
        const T* cf = coef + ((size_t)c * S + (size_t)W * w) * ncp + k;
        const T* xr = x + (size_t)clampi(pt.j + bb, 0, n - 1) * n;
        T cv[W], xv[W];
#pragma unroll
        for (int a = 0; a < W; ++a) cv[a] = stream_load(cf + (size_t)a * ncp);
#pragma unroll
        for (int a = 0; a < W; ++a) xv[a] = xr[clampi(pt.i + a - P, 0, n - 1)];
        T acc = 0;
#pragma unroll
        for (int a = 0; a < W; ++a) acc = fma(cv[a], xv[a], acc);
        if (w == P) diag = cv[P];
        return acc;
    }
};

template <int P, typename T_>
struct Kron2D {
    using T = T_;
    using Pt = Pt2;
    static constexpr int W = 2 * P + 1, NC = (P + 1) * (P + 1);
    static constexpr bool kColourOrder = false;
    const T* __restrict__ K;  // n x W bands
    const T* __restrict__ M;
    int n;
    int ncp;

    __device__ __forceinline__ int colour_size(int c) const {
        int ci = c % (P + 1), cj = c / (P + 1);
        return ((n - ci + P) / (P + 1)) * ((n - cj + P) / (P + 1));
    }
    __device__ __forceinline__ bool point(int c, int k, Pt& pt) const {
        int ci = c % (P + 1), cj = c / (P + 1);
        int ni = (n - ci + P) / (P + 1), nj = (n - cj + P) / (P + 1);
        if (k >= ni * nj) return false;
        int jj = k / ni, ii = k - jj * ni;
        pt.i = ci + (P + 1) * ii;
        pt.j = cj + (P + 1) * jj;
        pt.I = pt.i + (long long)n * pt.j;
        return true;
    }
    __device__ __forceinline__ bool point_nat(long long I, Pt& pt) const {
        if (I >= (long long)n * n) return false;
        pt.j = (int)(I / n);
        pt.i = (int)(I - (long long)pt.j * n);
        pt.I = I;
        return true;
    }
    static constexpr int NW = W;
    // Row bb = w - P of the sum-factorised product: M_jb (K_i . x_row) + K_jb (M_i . x_row).
    __device__ __forceinline__ T slice(const T* __restrict__ x, const Pt& pt, int, int, int w,
                                       T& diag) const {
        const int bb = w - P;
        const T* xr = x + (size_t)clampi(pt.j + bb, 0, n - 1) * n;
        T ki[W], mi[W], xv[W];
#pragma unroll
        for (int a = 0; a < W; ++a) {
            ki[a] = K[(size_t)pt.i * W + a];
            mi[a] = M[(size_t)pt.i * W + a];
            xv[a] = xr[clampi(pt.i + a - P, 0, n - 1)];
        }
        T mj = M[(size_t)pt.j * W + w], kj = K[(size_t)pt.j * W + w];
        T sk = 0, sm = 0;
#pragma unroll
        for (int a = 0; a < W; ++a) {
            sk = fma(ki[a], xv[a], sk);
            sm = fma(mi[a], xv[a], sm);
        }
        if (w == P) diag = ki[P] * mj + mi[P] * kj;
        return fma(mj, sk, kj * sm);
    }
};

template <int P, typename T_>
struct Kron3D {
    using T = T_;
    using Pt = Pt3;
    static constexpr int W = 2 * P + 1, NC = (P + 1) * (P + 1) * (P + 1);
    static constexpr bool kColourOrder = false;
    const T* __restrict__ K;
    const T* __restrict__ M;
    int n;
    int ncp;

    __device__ __forceinline__ int colour_size(int c) const {
        int ci = c % (P + 1), cj = (c / (P + 1)) % (P + 1), ck = c / ((P + 1) * (P + 1));
        return ((n - ci + P) / (P + 1)) * ((n - cj + P) / (P + 1)) * ((n - ck + P) / (P + 1));
    }
    __device__ __forceinline__ bool point(int c, int k, Pt& pt) const {
        int ci = c % (P + 1), cj = (c / (P + 1)) % (P + 1), ck = c / ((P + 1) * (P + 1));
        int ni = (n - ci + P) / (P + 1), nj = (n - cj + P) / (P + 1), nk = (n - ck + P) / (P + 1);
        if (k >= ni * nj * nk) return false;
        int kk = k / (ni * nj);
        int rem = k - kk * ni * nj;
        int jj = rem / ni, ii = rem - jj * ni;
        pt.i = ci + (P + 1) * ii;
        pt.j = cj + (P + 1) * jj;
        pt.k = ck + (P + 1) * kk;
        pt.I = pt.i + (long long)n * (pt.j + (long long)n * pt.k);
        return true;
    }
    __device__ __forceinline__ bool point_nat(long long I, Pt& pt) const {
        long long nn = (long long)n * n;
        if (I >= nn * n) return false;
        pt.k = (int)(I / nn);
        long long rem = I - (long long)pt.k * nn;
        pt.j = (int)(rem / n);
        pt.i = (int)(rem - (long long)pt.j * n);
        pt.I = I;
        return true;
    }
    static constexpr int NW = W;
    // Plane cc = w - P: M_kc (sum_b M_jb Kx + K_jb Mx) + K_kc (sum_b M_jb Mx).
    __device__ __forceinline__ T slice(const T* __restrict__ x, const Pt& pt, int, int, int w,
                                       T& diag) const {
        const int cc = w - P;
        T ki[W], mi[W], kj[W], mj[W];
#pragma unroll
        for (int a = 0; a < W; ++a) {
            ki[a] = K[(size_t)pt.i * W + a];
            mi[a] = M[(size_t)pt.i * W + a];
            kj[a] = K[(size_t)pt.j * W + a];
            mj[a] = M[(size_t)pt.j * W + a];
        }
        const size_t nn = (size_t)n * n;
        const T* xs = x + (size_t)clampi(pt.k + cc, 0, n - 1) * nn;
        T y1 = 0, y2 = 0;
#pragma unroll
        for (int bb = -P; bb <= P; ++bb) {
            const T* xr = xs + (size_t)clampi(pt.j + bb, 0, n - 1) * n;
            T xv[W];
#pragma unroll
            for (int a = 0; a < W; ++a) xv[a] = xr[clampi(pt.i + a - P, 0, n - 1)];
            T sk = 0, sm = 0;
#pragma unroll
            for (int a = 0; a < W; ++a) {
                sk = fma(ki[a], xv[a], sk);
                sm = fma(mi[a], xv[a], sm);
            }
            y1 = fma(mj[bb + P], sk, y1);
            y1 = fma(kj[bb + P], sm, y1);
            y2 = fma(mj[bb + P], sm, y2);
        }
        T mk = M[(size_t)pt.k * W + w], kk = K[(size_t)pt.k * W + w];
        if (w == P) diag = ki[P] * mj[P] * mk + mi[P] * kj[P] * mk + mi[P] * mj[P] * kk;
        return fma(mk, y1, kk * y2);
    }
};

// ---------------------------------------------------------------------------
// smoothing and residual kernels

// One colour of multicolour Gauss-Seidel: every point of colour c is updated
// from the values of x at the start of the pass (no two points of one colour
// are coupled, so the update order inside the pass is irrelevant):
// x_I <- x_I + (b_I - (A x)_I) / A_II.
// Layout: a block holds 64 points (one per lane) and Op::NW waves;
// wave w computes the partial product of stencil slice w for its 64 points
// (all of the slice's loads in flight at once), the partials meet in LDS and
// are summed in slice order.
template <class Op>
__device__ __forceinline__ void gs_colour_body(const Op& A, const typename Op::T* __restrict__ b,
                                               typename Op::T* __restrict__ x, int c, int blk) {
    using T = typename Op::T;
    __shared__ T part[Op::NW][64];
    __shared__ T dg[64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int k = blk * 64 + lane;
    typename Op::Pt pt;
    bool ok = A.point(c, k, pt);
    T d = 1, sl = 0;
    if (ok) sl = A.slice(x, pt, c, k, w, d);
    part[w][lane] = sl;
    if (w == Op::NW / 2) dg[lane] = d;
    __syncthreads();
    if (w == 0 && ok) {
        T acc = 0;
#pragma unroll
        for (int v = 0; v < Op::NW; ++v) acc += part[v][lane];
        x[pt.I] = x[pt.I] + (b[pt.I] - acc) / dg[lane];
    }
}

template <class Op>
__global__ void __launch_bounds__(64 * Op::NW) k_gs_colour_sliced(Op A,
                                                                  const typename Op::T* __restrict__ b,
                                                                  typename Op::T* __restrict__ x,
                                                                  int c) {
    gs_colour_body(A, b, x, c, xcd_swizzle(blockIdx.x, gridDim.x));
}

template <class Op, typename Tout>
__device__ __forceinline__ void residual_body(const Op& A, const typename Op::T* __restrict__ b,
                                              const typename Op::T* __restrict__ x,
                                              Tout* __restrict__ out, int mode, double omega,
                                              long long N, double* __restrict__ partial, int blk,
                                              int slot) {
    using T = typename Op::T;
    __shared__ T part[Op::NW][64];
    __shared__ T dg[64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    typename Op::Pt pt;
    bool ok;
    int c = 0, k = 0;
    if constexpr (Op::kColourOrder) {
        int bpc = A.ncp / 64;
        c = blk / bpc;
        k = (blk - c * bpc) * 64 + lane;
        ok = (c < Op::NC) && A.point(c, k, pt);
    } else {
        long long I = (long long)blk * 64 + lane;
        ok = (I < N) && A.point_nat(I, pt);
    }
    T d = 1, sl = 0;
    if (ok) sl = A.slice(x, pt, c, k, w, d);
    part[w][lane] = sl;
    if (w == Op::NW / 2) dg[lane] = d;
    __syncthreads();
    double sq = 0.0;
    if (w == 0 && ok) {
        T acc = 0;
#pragma unroll
        for (int v = 0; v < Op::NW; ++v) acc += part[v][lane];
        T v;
        if (mode == 0)
            v = b[pt.I] - acc;
        else if (mode == 1)
            v = acc;
        else
            v = x[pt.I] + (T)omega * (b[pt.I] - acc) / dg[lane];
        out[pt.I] = (Tout)v;
        sq = (double)v * (double)v;
    }
    if (partial) {
        if (w == 0) {
            double t = wave_sum(sq);
            if (lane == 0) partial[slot] = t;
        }
    }
}

// Residual-type products with the sliced layout: r = b - A x (mode 0),
// y = A x (mode 1), damped Jacobi step (mode 2); optional per-block sums of
// squares.  Colour-ordered traversal for stored stencils, natural otherwise.
template <class Op, typename Tout>
__global__ void __launch_bounds__(64 * Op::NW) k_residual_sliced(
    Op A, const typename Op::T* __restrict__ b, const typename Op::T* __restrict__ x,
    Tout* __restrict__ out, int mode, double omega, long long N, double* __restrict__ partial) {
    residual_body<Op, Tout>(A, b, x, out, mode, omega, N, partial, xcd_swizzle(blockIdx.x, gridDim.x),
                            blockIdx.x);
}

// Lexicographic Gauss-Seidel sweep (x index fastest, forward) in exact
// lexicographic semantics by one workgroup: point (i, j) only reads updated
// values of points before it in lexicographic order and within reach p, all of
// which lie on hyperplanes i + (p+1) j of smaller index, while the points after
// it lie on larger ones; the points of one hyperplane are therefore updated
// together, hyperplane after hyperplane.  Each row's slices are spread over
// the block's waves (2D operators).
constexpr int kLexThreads = 1024;
template <class Op>
__global__ void __launch_bounds__(kLexThreads) k_lexgs_sweep(Op A, const typename Op::T* __restrict__ b,
                                                             typename Op::T* __restrict__ x) {
    using T = typename Op::T;
    constexpr int P = (Op::NW - 1) / 2;
    constexpr int NW = Op::NW;
    constexpr int PPB = kLexThreads / 64 / NW;  // 64-point groups per pass
    __shared__ T part[PPB][NW][64];
    __shared__ T dg[PPB][64];
    const int n = A.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = wave / NW, w = wave % NW;
    const int tmax = (n - 1) + (P + 1) * (n - 1);
    for (int t = 0; t <= tmax; ++t) {
        int j0 = max(0, (t - (n - 1) + P) / (P + 1));
        int j1 = min(n - 1, t / (P + 1));
        int cnt = j1 - j0 + 1;
        for (int base = 0; base < cnt; base += PPB * 64) {
            int q = base + grp * 64 + lane;
            bool ok = grp < PPB && q < cnt;
            Pt2 pt;
            int c = 0, k = 0;
            T d = 1, sl = 0;
            if (ok) {
                pt.j = j0 + q;
                pt.i = t - (P + 1) * pt.j;
                pt.I = pt.i + (long long)n * pt.j;
                int ci = pt.i % (P + 1), cj = pt.j % (P + 1);
                c = ci + (P + 1) * cj;
                k = pt.i / (P + 1) + ((n - ci + P) / (P + 1)) * (pt.j / (P + 1));
                sl = A.slice(x, pt, c, k, w, d);
            }
            if (grp < PPB) {
                part[grp][w][lane] = sl;
                if (w == NW / 2) dg[grp][lane] = d;
            }
            __syncthreads();
            if (ok && w == 0) {
                T acc = 0;
#pragma unroll
                for (int v = 0; v < NW; ++v) acc += part[grp][v][lane];
                x[pt.I] = x[pt.I] + (b[pt.I] - acc) / dg[grp][lane];
            }
            __syncthreads();
        }
    }
}

// Deterministic final reduction: out[0] = sqrt(sum partial) / denom.
__global__ void __launch_bounds__(kBlock) k_finalize_norm(const double* __restrict__ partial,
                                                          int np, double denom,
                                                          const double* __restrict__ denom_dev,
                                                          double* __restrict__ out) {
    __shared__ double red[kBlock / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) s += partial[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        double d = denom_dev ? *denom_dev : denom;
        out[0] = sqrt(s) / d;
    }
}

// Per-block sums of squares of a vector.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sumsq(const T* __restrict__ v, long long N,
                                                  double* __restrict__ partial) {
    __shared__ double red[kBlock / 64];
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    double s = 0.0;
    for (; I < N; I += (long long)gridDim.x * kBlock) {
        double t = (double)v[I];
        s += t * t;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// elementwise kernels

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBlock) k_copy(const Tin* __restrict__ a, Tout* __restrict__ b,
                                                 long long N) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I < N) b[I] = (Tout)a[I];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ a, T v, long long N) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I < N) a[I] = v;
}

// x64 += e32 (refinement update)
__global__ void __launch_bounds__(kBlock) k_add_f32_to_f64(const float* __restrict__ e,
                                                           double* __restrict__ x, long long N) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I < N) x[I] += (double)e[I];
}

// ---------------------------------------------------------------------------
// transfers (R = P^T, P = P1 (x) P1 [(x) P1])

// bc = R rf on the coarse grid; xc (if given) is zeroed: the coarse-grid
// correction of Algorithm 2 starts from a zero error.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict2d(const T* __restrict__ rf, int nf,
                                                       T* __restrict__ bc, int nc,
                                                       const int* __restrict__ rs,
                                                       const T* __restrict__ rw, int RW,
                                                       T* __restrict__ xc) {
    long long C = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (C >= (long long)nc * nc) return;
    if (xc) xc[C] = 0;
    int J = (int)(C / nc), I = (int)(C - (long long)J * nc);
    int si = rs[I], sj = rs[J];
    T acc = 0;
    for (int b = 0; b < RW; ++b) {
        T wj = rw[(size_t)J * RW + b];
        const T* row = rf + (size_t)min(sj + b, nf - 1) * nf;
        T s = 0;
        for (int a = 0; a < RW; ++a) s = fma(rw[(size_t)I * RW + a], row[min(si + a, nf - 1)], s);
        acc = fma(wj, s, acc);
    }
    bc[C] = acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong2d(const T* __restrict__ ec, int nc,
                                                      T* __restrict__ xf, int nf,
                                                      const int* __restrict__ ps,
                                                      const T* __restrict__ pw, int PW) {
    long long F = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (F >= (long long)nf * nf) return;
    int j = (int)(F / nf), i = (int)(F - (long long)j * nf);
    int si = ps[i], sj = ps[j];
    T acc = 0;
    for (int b = 0; b < PW; ++b) {
        T wj = pw[(size_t)j * PW + b];
        const T* row = ec + (size_t)min(sj + b, nc - 1) * nc;
        T s = 0;
        for (int a = 0; a < PW; ++a) s = fma(pw[(size_t)i * PW + a], row[min(si + a, nc - 1)], s);
        acc = fma(wj, s, acc);
    }
    xf[F] += acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict3d(const T* __restrict__ rf, int nf,
                                                       T* __restrict__ bc, int nc,
                                                       const int* __restrict__ rs,
                                                       const T* __restrict__ rw, int RW,
                                                       T* __restrict__ xc) {
    long long C = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long ncc = (long long)nc * nc;
    if (C >= ncc * nc) return;
    if (xc) xc[C] = 0;
    int K = (int)(C / ncc);
    long long rem = C - (long long)K * ncc;
    int J = (int)(rem / nc), I = (int)(rem - (long long)J * nc);
    int si = rs[I], sj = rs[J], sk = rs[K];
    T acc = 0;
    for (int c = 0; c < RW; ++c) {
        T wk = rw[(size_t)K * RW + c];
        const T* sl = rf + (size_t)min(sk + c, nf - 1) * nf * nf;
        T s2 = 0;
        for (int b = 0; b < RW; ++b) {
            T wj = rw[(size_t)J * RW + b];
            const T* row = sl + (size_t)min(sj + b, nf - 1) * nf;
            T s = 0;
            for (int a = 0; a < RW; ++a)
                s = fma(rw[(size_t)I * RW + a], row[min(si + a, nf - 1)], s);
            s2 = fma(wj, s, s2);
        }
        acc = fma(wk, s2, acc);
    }
    bc[C] = acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong3d(const T* __restrict__ ec, int nc,
                                                      T* __restrict__ xf, int nf,
                                                      const int* __restrict__ ps,
                                                      const T* __restrict__ pw, int PW) {
    long long F = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long nff = (long long)nf * nf;
    if (F >= nff * nf) return;
    int k = (int)(F / nff);
    long long rem = F - (long long)k * nff;
    int j = (int)(rem / nf), i = (int)(rem - (long long)j * nf);
    int si = ps[i], sj = ps[j], sk = ps[k];
    T acc = 0;
    for (int c = 0; c < PW; ++c) {
        T wk = pw[(size_t)k * PW + c];
        const T* sl = ec + (size_t)min(sk + c, nc - 1) * nc * nc;
        T s2 = 0;
        for (int b = 0; b < PW; ++b) {
            T wj = pw[(size_t)j * PW + b];
            const T* row = sl + (size_t)min(sj + b, nc - 1) * nc;
            T s = 0;
            for (int a = 0; a < PW; ++a)
                s = fma(pw[(size_t)i * PW + a], row[min(si + a, nc - 1)], s);
            s2 = fma(wj, s, s2);
        }
        acc = fma(wk, s2, acc);
    }
    xf[F] += acc;
}

// Coarsest grid: x = A_0^{-1} b with the inverse formed from the FP64 Cholesky
// factor at setup; accumulated in FP64 for either precision.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_solve(const double* __restrict__ Ainv, int nc,
                                                         const T* __restrict__ b,
                                                         T* __restrict__ x) {
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < nc; r += gridDim.x * kBlock) {
        double s = 0.0;
        for (int c = 0; c < nc; ++c) s = fma(Ainv[(size_t)r * nc + c], (double)b[c], s);
        x[r] = (T)s;
    }
}

// ---------------------------------------------------------------------------
// extrapolation: tall-skinny QR of Delta S = [s_1 - s_0, ..., s_{q+1} - s_q]

// Householder QR of an m x n panel held column-major in LDS (a[col*m + row]);
// writes the n x n R factor (row-major) to R.  Rows are distributed over the
// block; the two reductions per column use the deterministic block_sum.
__device__ inline void panel_qr(double* a, int m, int n, double* R, double* red) {
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int r = k + threadIdx.x; r < m; r += blockDim.x) s += a[k * m + r] * a[k * m + r];
        s = block_sum(s, red);
        double akk = a[k * m + k];
        double nrm = sqrt(s);
        __syncthreads();
        if (nrm == 0.0) {
            if (threadIdx.x == 0) {
                R[k * n + k] = 0.0;
                for (int j = k + 1; j < n; ++j) R[k * n + j] = a[j * m + k];
            }
            __syncthreads();
            continue;
        }
        double alpha = akk > 0.0 ? -nrm : nrm;
        double vk = akk - alpha;
        double vtv = s - akk * akk + vk * vk;
        if (threadIdx.x == 0) a[k * m + k] = vk;
        __syncthreads();
        for (int j = k + 1; j < n; ++j) {
            double w = 0.0;
            for (int r = k + threadIdx.x; r < m; r += blockDim.x) w += a[k * m + r] * a[j * m + r];
            w = block_sum(w, red);
            double f = 2.0 * w / vtv;
            for (int r = k + threadIdx.x; r < m; r += blockDim.x) a[j * m + r] -= f * a[k * m + r];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            R[k * n + k] = alpha;
            for (int j = k + 1; j < n; ++j) R[k * n + j] = a[j * m + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < k; ++j) R[k * n + j] = 0.0;
}

// Leaf: panel of kQrRows consecutive unknowns, columns s_{j+1} - s_j.
__global__ void __launch_bounds__(kBlock) k_tsqr_leaf(IterPtrs S, int ncols, long long N,
                                                      double* __restrict__ Rout) {
    extern __shared__ double lds[];
    __shared__ double red[kBlock / 64];
    double* a = lds;
    const int m = kQrRows;
    long long base = (long long)blockIdx.x * m;
    for (int r = threadIdx.x; r < m; r += kBlock) {
        long long I = base + r;
        bool in = I < N;
        double prev = in ? S.s[0][I] : 0.0;
        for (int j = 0; j < ncols; ++j) {
            double nxt = in ? S.s[j + 1][I] : 0.0;
            a[j * m + r] = nxt - prev;
            prev = nxt;
        }
    }
    __syncthreads();
    __shared__ double Rl[kMaxCols * kMaxCols];
    panel_qr(a, m, ncols, Rl, red);
    __syncthreads();
    for (int t = threadIdx.x; t < ncols * ncols; t += kBlock)
        Rout[(size_t)blockIdx.x * ncols * ncols + t] = Rl[t];
}

// Inner node: stack up to `group` R factors of the previous level and QR them.
__global__ void __launch_bounds__(kBlock) k_tsqr_node(const double* __restrict__ Rin, int count,
                                                      int group, int ncols,
                                                      double* __restrict__ Rout) {
    extern __shared__ double lds[];
    __shared__ double red[kBlock / 64];
    const int m = group * ncols;
    double* a = lds;
    int first = blockIdx.x * group;
    for (int t = threadIdx.x; t < m * ncols; t += kBlock) {
        int j = t / m, r = t - j * m;   // column j, stacked row r
        int child = first + r / ncols, rr = r % ncols;
        a[t] = (child < count) ? Rin[(size_t)child * ncols * ncols + rr * ncols + j] : 0.0;
    }
    __syncthreads();
    __shared__ double Rl[kMaxCols * kMaxCols];
    panel_qr(a, m, ncols, Rl, red);
    __syncthreads();
    for (int t = threadIdx.x; t < ncols * ncols; t += kBlock)
        Rout[(size_t)blockIdx.x * ncols * ncols + t] = Rl[t];
}

// Coefficients gamma of Algorithm 3 (RRE: R^T R d = 1) or Algorithm 4 (MPE:
// R_q d = -r_q, d_q = 1), gamma = d / sum(d), alpha_j = 1 - sum_{i<=j} gamma_i.
// Breakdown rules: first column j with |R_jj| <= 1e-13 ||R_{:,j}|| -> use
// columns 0..j with d = (-R_{<j}^{-1} R_{<j,j}, 1) (exact for a linear map);
// |sum d| <= 1e-14 ||d||_1 -> info = -1 (no extrapolation).
__global__ void k_extrap_coeffs(const double* __restrict__ Rg, int ncols, int method,
                                ExtrapCoeffs* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double R[kMaxCols][kMaxCols], d[kMaxCols], y[kMaxCols];
    const int n = ncols, q = ncols - 1;
    bool finite = true;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            R[i][j] = Rg[i * n + j];
            if (!isfinite(R[i][j])) finite = false;
        }
    ExtrapCoeffs c;
    for (int i = 0; i < kMaxCols; ++i) c.gamma[i] = c.alpha[i] = 0.0;
    c.info = 0;
    c.lucky_col = -1;
    if (!finite) {
        c.info = -2;
        *out = c;
        return;
    }
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    int lucky = -1;
    for (int j = 0; j < n && lucky < 0; ++j) {
        double cn = 0.0;
        for (int i = 0; i <= j; ++i) cn += R[i][j] * R[i][j];
        if (fabs(R[j][j]) <= 1e-13 * sqrt(cn)) lucky = j;
    }
    if (lucky == 0) {
        d[0] = 1.0;
        c.info = 1;
    } else if (lucky > 0) {
        for (int i = lucky - 1; i >= 0; --i) {
            double s = -R[i][lucky];
            for (int k = i + 1; k < lucky; ++k) s -= R[i][k] * d[k];
            d[i] = s / R[i][i];
        }
        d[lucky] = 1.0;
        c.info = 1;
    } else if (method == 1) {  // RRE: R^T y = 1, R d = y
        for (int i = 0; i < n; ++i) {
            double s = 1.0;
            for (int k = 0; k < i; ++k) s -= R[k][i] * y[k];
            y[i] = s / R[i][i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= R[i][k] * d[k];
            d[i] = s / R[i][i];
        }
    } else {  // MPE
        for (int i = q - 1; i >= 0; --i) {
            double s = -R[i][q];
            for (int k = i + 1; k < q; ++k) s -= R[i][k] * d[k];
            d[i] = s / R[i][i];
        }
        d[q] = 1.0;
    }
    c.lucky_col = lucky;
    double lam = 0.0, l1 = 0.0;
    for (int i = 0; i < n; ++i) {
        lam += d[i];
        l1 += fabs(d[i]);
    }
    if (!isfinite(lam) || fabs(lam) <= 1e-14 * l1) {
        c.info = -1;
        *out = c;
        return;
    }
    double acc = 1.0;
    for (int i = 0; i < n; ++i) c.gamma[i] = d[i] / lam;
    for (int j = 0; j < q; ++j) {
        acc -= c.gamma[j];
        c.alpha[j] = acc;
    }
    *out = c;
}

// t = s_0 + sum_{j<q} alpha_j (s_{j+1} - s_j); on breakdown t = s_{q+1}.
// `out` may alias s_0.
__global__ void __launch_bounds__(kBlock) k_extrap_combine(IterPtrs S, int q, long long N,
                                                           const ExtrapCoeffs* __restrict__ cf,
                                                           double* out) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I >= N) return;
    int info = cf->info;
    if (info < 0) {
        out[I] = S.s[q + 1][I];
        return;
    }
    double prev = S.s[0][I];
    double t = prev;
    for (int j = 0; j < q; ++j) {
        double nxt = S.s[j + 1][I];
        t = fma(cf->alpha[j], nxt - prev, t);
        prev = nxt;
    }
    out[I] = t;
}


// ---------------------------------------------------------------------------
// single-workgroup V-cycle on the small levels 0..top (one launch replaces the
// hundreds of tiny launches those levels would need; colour passes are
// separated by workgroup barriers and the data stay in L2)

constexpr int kTailMaxLevels = 8;
constexpr int kTailThreads = 1024;
constexpr int kTailMaxChunks = 8;  // 64-point chunks held in LDS at once

template <class Op>
struct TailArgs {
    using T = typename Op::T;
    int top;                        // finest level handled here
    int nu1, nu2;
    int n0;                         // coarsest unknowns
    const double* Ainv;             // coarsest inverse (FP64)
    Op op[kTailMaxLevels];
    long long N[kTailMaxLevels];
    T* x[kTailMaxLevels];
    T* b[kTailMaxLevels];
    T* r[kTailMaxLevels];
    const int* rs[kTailMaxLevels];  // transfer tables between l-1 and l
    const T* rw[kTailMaxLevels];
    const int* ps[kTailMaxLevels];
    const T* pw[kTailMaxLevels];
    int RW[kTailMaxLevels], PW[kTailMaxLevels];
};

// One colour pass (mode 0) or residual of colour c (mode 1, into r) by the
// whole block, sliced as in the multi-block kernels.
template <class Op>
__device__ void tail_colour(const Op& A, const typename Op::T* b, typename Op::T* x,
                            typename Op::T* r, int c, int mode, typename Op::T* part,
                            typename Op::T* dg) {
    using T = typename Op::T;
    constexpr int NW = Op::NW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = kTailThreads / 64;
    const int cs = A.colour_size(c);
    for (int ch0 = 0; ch0 * 64 < cs; ch0 += kTailMaxChunks) {
        int nch = min(kTailMaxChunks, (cs + 63) / 64 - ch0);
        for (int it = wave; it < nch * NW; it += nwave) {
            int ch = it / NW, w = it - ch * NW;
            int k = (ch0 + ch) * 64 + lane;
            typename Op::Pt pt;
            T d = 1, sl = 0;
            if (A.point(c, k, pt)) sl = A.slice(x, pt, c, k, w, d);
            part[(ch * NW + w) * 64 + lane] = sl;
            if (w == NW / 2) dg[ch * 64 + lane] = d;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < nch * 64; t += kTailThreads) {
            int ch = t >> 6, ln = t & 63;
            int k = (ch0 + ch) * 64 + ln;
            typename Op::Pt pt;
            if (!A.point(c, k, pt)) continue;
            T acc = 0;
#pragma unroll
            for (int v = 0; v < NW; ++v) acc += part[(ch * NW + v) * 64 + ln];
            if (mode == 0)
                x[pt.I] = x[pt.I] + (b[pt.I] - acc) / dg[t];
            else
                r[pt.I] = b[pt.I] - acc;
        }
        __syncthreads();
    }
}

template <typename T>
__device__ void tail_restrict(const T* rf, int nf, T* bc, T* xc, int nc, const int* rs,
                              const T* rw, int RW, int dim) {
    long long Nc = (long long)nc * nc * (dim == 3 ? nc : 1);
    for (long long C = threadIdx.x; C < Nc; C += kTailThreads) {
        int I = (int)(C % nc), J = (int)((C / nc) % nc), K = (dim == 3) ? (int)(C / ((long long)nc * nc)) : 0;
        T acc = 0;
        int KR = (dim == 3) ? RW : 1;
        for (int cc = 0; cc < KR; ++cc) {
            T wk = (dim == 3) ? rw[(size_t)K * RW + cc] : (T)1;
            size_t zoff = (dim == 3) ? (size_t)min(rs[K] + cc, nf - 1) * nf * nf : 0;
            T s2 = 0;
            for (int bq = 0; bq < RW; ++bq) {
                const T* row = rf + zoff + (size_t)min(rs[J] + bq, nf - 1) * nf;
                T s1 = 0;
                for (int a = 0; a < RW; ++a) s1 = fma(rw[(size_t)I * RW + a], row[min(rs[I] + a, nf - 1)], s1);
                s2 = fma(rw[(size_t)J * RW + bq], s1, s2);
            }
            acc = fma(wk, s2, acc);
        }
        bc[C] = acc;
        xc[C] = 0;
    }
}

template <typename T>
__device__ void tail_prolong(const T* ec, int nc, T* xf, int nf, const int* ps, const T* pw,
                             int PW, int dim) {
    long long Nf = (long long)nf * nf * (dim == 3 ? nf : 1);
    for (long long F = threadIdx.x; F < Nf; F += kTailThreads) {
        int i = (int)(F % nf), j = (int)((F / nf) % nf), k = (dim == 3) ? (int)(F / ((long long)nf * nf)) : 0;
        T acc = 0;
        int KP = (dim == 3) ? PW : 1;
        for (int cc = 0; cc < KP; ++cc) {
            T wk = (dim == 3) ? pw[(size_t)k * PW + cc] : (T)1;
            size_t zoff = (dim == 3) ? (size_t)min(ps[k] + cc, nc - 1) * nc * nc : 0;
            T s2 = 0;
            for (int bq = 0; bq < PW; ++bq) {
                const T* row = ec + zoff + (size_t)min(ps[j] + bq, nc - 1) * nc;
                T s1 = 0;
                for (int a = 0; a < PW; ++a) s1 = fma(pw[(size_t)i * PW + a], row[min(ps[i] + a, nc - 1)], s1);
                s2 = fma(pw[(size_t)j * PW + bq], s1, s2);
            }
            acc = fma(wk, s2, acc);
        }
        xf[F] += acc;
    }
}

// V-cycle (Algorithm 2, mu = 1) on levels 0..top with right-hand side b[top]
// and iterate x[top] (in place), by one workgroup.
template <class Op>
__device__ void vcycle_tail_body(const TailArgs<Op>& a) {
    using T = typename Op::T;
    constexpr int NW = Op::NW;
    constexpr int DIM = std::is_same<typename Op::Pt, Pt3>::value ? 3 : 2;
    __shared__ T part[kTailMaxChunks * NW * 64];
    __shared__ T dg[kTailMaxChunks * 64];
    for (int l = a.top; l >= 1; --l) {
        const Op& A = a.op[l];
        for (int s = 0; s < a.nu1; ++s)
            for (int c = 0; c < Op::NC; ++c) tail_colour(A, a.b[l], a.x[l], a.r[l], c, 0, part, dg);
        for (int c = 0; c < Op::NC; ++c) tail_colour(A, a.b[l], a.x[l], a.r[l], c, 1, part, dg);
        tail_restrict(a.r[l], A.n, a.b[l - 1], a.x[l - 1], a.op[l - 1].n, a.rs[l], a.rw[l], a.RW[l], DIM);
        __syncthreads();
    }
    for (int r = threadIdx.x; r < a.n0; r += kTailThreads) {
        double s = 0.0;
        for (int c = 0; c < a.n0; ++c) s = fma(a.Ainv[(size_t)r * a.n0 + c], (double)a.b[0][c], s);
        a.x[0][r] = (T)s;
    }
    __syncthreads();
    for (int l = 1; l <= a.top; ++l) {
        const Op& A = a.op[l];
        tail_prolong(a.x[l - 1], a.op[l - 1].n, a.x[l], A.n, a.ps[l], a.pw[l], a.PW[l], DIM);
        __syncthreads();
        for (int s = 0; s < a.nu2; ++s)
            for (int c = 0; c < Op::NC; ++c) tail_colour(A, a.b[l], a.x[l], a.r[l], c, 0, part, dg);
    }
}

template <class Op>
__global__ void __launch_bounds__(kTailThreads) k_vcycle_tail(TailArgs<Op> a) {
    vcycle_tail_body(a);
}

// Batched: workgroup e runs problem e's small-level V-cycle.
template <class Op>
__global__ void __launch_bounds__(kTailThreads) k_b_tail(const TailArgs<Op>* __restrict__ A) {
    vcycle_tail_body(A[blockIdx.x]);
}

// ---------------------------------------------------------------------------
// setup kernels (FP64): mapped assembly of the finest stencil, load vector,
// Galerkin products on stencils, colour-blocked layout

// Quarter annulus as the degree-2 B-spline surface on one element with control
// net rho_a * {(1,0), (1,1), (0,1)}_b, rho = (1, 1.5, 2).  At every quadrature
// point stores w |det J| (J^T J)^{-1} (3 entries) and w |det J| (for loads) and
// the physical point.
struct GeomQP {
    double* D11;
    double* D12;
    double* D22;
    double* wdet;
    double* X;
    double* Y;
};

__device__ inline void bernstein2(double u, double* B, double* dB) {
    B[0] = (1 - u) * (1 - u);
    B[1] = 2 * u * (1 - u);
    B[2] = u * u;
    dB[0] = -2 * (1 - u);
    dB[1] = 2 - 4 * u;
    dB[2] = 2 * u;
}

__global__ void k_geometry_qp(int geom, int NQ, const double* __restrict__ pts,
                              const double* __restrict__ wts, GeomQP G) {
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)NQ * NQ) return;
    int qy = (int)(t / NQ), qx = (int)(t - (long long)qy * NQ);
    double xi = pts[qx], eta = pts[qy];
    double J00, J01, J10, J11, X, Y;
    if (geom == 1) {
        const double rho[3] = {1.0, 1.5, 2.0};
        const double cx[3] = {1.0, 1.0, 0.0}, cy[3] = {0.0, 1.0, 1.0};
        double Bu[3], dBu[3], Bv[3], dBv[3];
        bernstein2(xi, Bu, dBu);
        bernstein2(eta, Bv, dBv);
        X = Y = J00 = J01 = J10 = J11 = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double px = rho[a] * cx[b], py = rho[a] * cy[b];
                X += Bu[a] * Bv[b] * px;
                Y += Bu[a] * Bv[b] * py;
                J00 += dBu[a] * Bv[b] * px;
                J01 += Bu[a] * dBv[b] * px;
                J10 += dBu[a] * Bv[b] * py;
                J11 += Bu[a] * dBv[b] * py;
            }
    } else {
        X = xi;
        Y = eta;
        J00 = 1.0;
        J01 = 0.0;
        J10 = 0.0;
        J11 = 1.0;
    }
    double det = J00 * J11 - J01 * J10;
    double a = J00 * J00 + J10 * J10, b = J00 * J01 + J10 * J11, c = J01 * J01 + J11 * J11;
    double w = wts[qx] * wts[qy] * fabs(det);
    double id = 1.0 / (a * c - b * b);
    G.D11[t] = w * c * id;
    G.D12[t] = -w * b * id;
    G.D22[t] = w * a * id;
    G.wdet[t] = w;
    G.X[t] = X;
    G.Y[t] = Y;
}

// Row-gather assembly of the finest stencil: entry (I, o) sums over the
// elements shared by functions I and I+o and their Gauss points.
// V/D: per flat 1D quadrature point, the p+1 local basis values/derivatives.
template <int P>
__global__ void k_assemble_stencil(int ne, int nq, const double* __restrict__ V,
                                   const double* __restrict__ D, GeomQP G,
                                   double* __restrict__ out) {
    constexpr int W = 2 * P + 1, S = W * W;
    const int n = ne + P - 2;
    const int NQ = ne * nq;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)n * n * S) return;
    long long I = t / S;
    int o = (int)(t - I * S);
    int j = (int)(I / n), i = (int)(I - (long long)j * n);
    int da = o % W - P, db = o / W - P;
    int i2 = i + da, j2 = j + db;
    double acc = 0.0;
    if (i2 >= 0 && i2 < n && j2 >= 0 && j2 < n) {
        // global function indices (Dirichlet function 0 removed)
        int gi = i + 1, gi2 = i2 + 1, gj = j + 1, gj2 = j2 + 1;
        int ex0 = max(max(gi, gi2) - P, 0), ex1 = min(min(gi, gi2), ne - 1);
        int ey0 = max(max(gj, gj2) - P, 0), ey1 = min(min(gj, gj2), ne - 1);
        for (int ey = ey0; ey <= ey1; ++ey)
            for (int qy = 0; qy < nq; ++qy) {
                int fy = ey * nq + qy;
                double vj = V[(size_t)fy * (P + 1) + gj - ey], dj = D[(size_t)fy * (P + 1) + gj - ey];
                double vj2 = V[(size_t)fy * (P + 1) + gj2 - ey], dj2 = D[(size_t)fy * (P + 1) + gj2 - ey];
                for (int ex = ex0; ex <= ex1; ++ex)
                    for (int qx = 0; qx < nq; ++qx) {
                        int fx = ex * nq + qx;
                        double vi = V[(size_t)fx * (P + 1) + gi - ex], di = D[(size_t)fx * (P + 1) + gi - ex];
                        double vi2 = V[(size_t)fx * (P + 1) + gi2 - ex],
                               di2 = D[(size_t)fx * (P + 1) + gi2 - ex];
                        size_t qi = (size_t)fy * NQ + fx;
                        double gx1 = di * vj, gy1 = vi * dj;   // reference gradient of I
                        double gx2 = di2 * vj2, gy2 = vi2 * dj2;
                        acc += G.D11[qi] * gx1 * gx2 + G.D12[qi] * (gx1 * gy2 + gy1 * gx2) +
                               G.D22[qi] * gy1 * gy2;
                    }
            }
    }
    out[t] = acc;
}

// f at the quadrature points: f = sum_m a_m sin(pi (k_m x + l_m y) + phi_m),
// stored premultiplied by w |det J|.
__global__ void k_load_qp(long long nqp, GeomQP G, const double* __restrict__ modes, int n_modes,
                          double* __restrict__ fq) {
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nqp) return;
    double X = G.X[t], Y = G.Y[t], f = 0.0;
    for (int m = 0; m < n_modes; ++m) {
        const double* md = modes + 4 * m;
        f += md[0] * sin(M_PI * (md[1] * X + md[2] * Y) + md[3]);
    }
    fq[t] = f * G.wdet[t];
}

// b_I = sum over the support of I and its Gauss points of (w |det J| f) phi_I.
__global__ void k_assemble_load2d(int ne, int p, int nq, const double* __restrict__ V,
                                  const double* __restrict__ fq, double* __restrict__ b) {
    const int n = ne + p - 2;
    const int NQ = ne * nq;
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I >= (long long)n * n) return;
    int j = (int)(I / n), i = (int)(I - (long long)j * n);
    int gi = i + 1, gj = j + 1;
    double acc = 0.0;
    for (int ey = max(gj - p, 0); ey <= min(gj, ne - 1); ++ey)
        for (int qy = 0; qy < nq; ++qy) {
            int fy = ey * nq + qy;
            double vj = V[(size_t)fy * (p + 1) + gj - ey];
            for (int ex = max(gi - p, 0); ex <= min(gi, ne - 1); ++ex)
                for (int qx = 0; qx < nq; ++qx) {
                    int fx = ex * nq + qx;
                    acc += fq[(size_t)fy * NQ + fx] * V[(size_t)fx * (p + 1) + gi - ex] * vj;
                }
        }
    b[I] = acc;
}

// 3D unit-cube load vector with flat 1D quadrature tables (identity map):
// f = sum_m a_m sin(pi (k x + l y + m z) + phi), modes of 5 entries.
__global__ void k_assemble_load3d(int ne, int p, int nq, const double* __restrict__ V,
                                  const double* __restrict__ pts, const double* __restrict__ wts,
                                  const double* __restrict__ modes, int n_modes,
                                  double* __restrict__ b) {
    const int n = ne + p - 2;
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long nn = (long long)n * n;
    if (I >= nn * n) return;
    int k = (int)(I / nn);
    long long rem = I - (long long)k * nn;
    int j = (int)(rem / n), i = (int)(rem - (long long)j * n);
    int gi = i + 1, gj = j + 1, gk = k + 1;
    double acc = 0.0;
    for (int ez = max(gk - p, 0); ez <= min(gk, ne - 1); ++ez)
        for (int qz = 0; qz < nq; ++qz) {
            int fz = ez * nq + qz;
            double vz = V[(size_t)fz * (p + 1) + gk - ez] * wts[fz], Z = pts[fz];
            for (int ey = max(gj - p, 0); ey <= min(gj, ne - 1); ++ey)
                for (int qy = 0; qy < nq; ++qy) {
                    int fy = ey * nq + qy;
                    double vy = V[(size_t)fy * (p + 1) + gj - ey] * wts[fy], Yv = pts[fy];
                    for (int ex = max(gi - p, 0); ex <= min(gi, ne - 1); ++ex)
                        for (int qx = 0; qx < nq; ++qx) {
                            int fx = ex * nq + qx;
                            double Xv = pts[fx];
                            double f = 0.0;
                            for (int m = 0; m < n_modes; ++m) {
                                const double* md = modes + 5 * m;
                                f += md[0] * sin(M_PI * (md[1] * Xv + md[2] * Yv + md[3] * Z) + md[4]);
                            }
                            acc += f * V[(size_t)fx * (p + 1) + gi - ex] * wts[fx] * vy * vz;
                        }
                }
        }
    b[I] = acc;
}

// Galerkin product on stencils, x direction: rows (I, j) with I coarse and j fine,
// T[(I,j)][(a'+P) + W(b+P)] = sum_{i,i'} P1[i,I] A[(i,j)][(i'-i+P) + W(b+P)] P1[i',I+a'].
template <int P>
__global__ void k_rap_x(const double* __restrict__ A, int nf, int nc, const int* __restrict__ rs,
                        const double* __restrict__ rw, int RW, double* __restrict__ Tout) {
    constexpr int W = 2 * P + 1, S = W * W;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)nc * nf * S) return;
    long long row = t / S;
    int o = (int)(t - row * S);
    int j = (int)(row / nc), I = (int)(row - (long long)j * nc);
    int ap = o % W - P, b = o / W - P;
    int I2 = I + ap;
    double acc = 0.0;
    if (I2 >= 0 && I2 < nc) {
        for (int s = 0; s < RW; ++s) {
            double w1 = rw[(size_t)I * RW + s];
            if (w1 == 0.0) continue;
            int i = rs[I] + s;
            const double* Ar = A + ((size_t)i + (size_t)nf * j) * S;
            for (int u = 0; u < RW; ++u) {
                double w2 = rw[(size_t)I2 * RW + u];
                int i2 = rs[I2] + u;
                int d = i2 - i;
                if (w2 == 0.0 || d < -P || d > P) continue;
                acc += w1 * Ar[(d + P) + W * (b + P)] * w2;
            }
        }
    }
    Tout[t] = acc;
}

// y direction: A_c[(I,J)][(a'+P) + W(b'+P)] = sum_{j,j'} P1[j,J] T[(I,j)][(a'+P)+W(j'-j+P)] P1[j',J+b'].
template <int P>
__global__ void k_rap_y(const double* __restrict__ Tin, int nf, int nc, const int* __restrict__ rs,
                        const double* __restrict__ rw, int RW, double* __restrict__ Ac) {
    constexpr int W = 2 * P + 1, S = W * W;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)nc * nc * S) return;
    long long row = t / S;
    int o = (int)(t - row * S);
    int J = (int)(row / nc), I = (int)(row - (long long)J * nc);
    int ap = o % W - P, bp = o / W - P;
    int J2 = J + bp;
    double acc = 0.0;
    if (J2 >= 0 && J2 < nc && I + ap >= 0 && I + ap < nc) {
        for (int s = 0; s < RW; ++s) {
            double w1 = rw[(size_t)J * RW + s];
            if (w1 == 0.0) continue;
            int j = rs[J] + s;
            const double* Tr = Tin + ((size_t)I + (size_t)nc * j) * S;
            for (int u = 0; u < RW; ++u) {
                double w2 = rw[(size_t)J2 * RW + u];
                int j2 = rs[J2] + u;
                int d = j2 - j;
                if (w2 == 0.0 || d < -P || d > P) continue;
                acc += w1 * Tr[(ap + P) + W * (d + P)] * w2;
            }
        }
    }
    Ac[t] = acc;
}

// Natural row-major stencil rows -> colour-blocked FP64 and FP32 copies.
template <int P>
__global__ void k_to_colour_blocked(const double* __restrict__ st, int n, int ncp,
                                    double* __restrict__ c64, float* __restrict__ c32) {
    constexpr int W = 2 * P + 1, S = W * W;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)n * n * S) return;
    long long I = t / S;
    int o = (int)(t - I * S);
    int j = (int)(I / n), i = (int)(I - (long long)j * n);
    int ci = i % (P + 1), cj = j % (P + 1);
    int c = ci + (P + 1) * cj;
    int ni = (n - ci + P) / (P + 1);
    int k = i / (P + 1) + ni * (j / (P + 1));
    size_t dst = ((size_t)c * S + o) * ncp + k;
    double v = st[t];
    c64[dst] = v;
    if (c32) c32[dst] = (float)v;
}

// Unit-square Kronecker operator K(x)M + M(x)K written out as colour-blocked
// (2p+1)^2 stencils (FP64 and FP32), entry by entry from the band factors.
template <int P>
__global__ void k_kron_to_stencil(const double* __restrict__ K, const double* __restrict__ M, int n,
                                  int ncp, double* __restrict__ c64, float* __restrict__ c32) {
    constexpr int W = 2 * P + 1, S = W * W;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)n * n * S) return;
    long long I = t / S;
    int o = (int)(t - I * S);
    int j = (int)(I / n), i = (int)(I - (long long)j * n);
    int da = o % W - P, db = o / W - P;
    double v = 0.0;
    if (i + da >= 0 && i + da < n && j + db >= 0 && j + db < n)
        v = K[(size_t)i * W + da + P] * M[(size_t)j * W + db + P] +
            M[(size_t)i * W + da + P] * K[(size_t)j * W + db + P];
    int ci = i % (P + 1), cj = j % (P + 1);
    int c = ci + (P + 1) * cj;
    int ni = (n - ci + P) / (P + 1);
    int k = i / (P + 1) + ni * (j / (P + 1));
    size_t dst = ((size_t)c * S + o) * ncp + k;
    c64[dst] = v;
    c32[dst] = (float)v;
}

// Diagonal of a colour-blocked stencil in natural order (FP64 and FP32).
template <int P>
__global__ void k_diag_stencil(const double* __restrict__ c64, int n, int ncp,
                               double* __restrict__ d64, float* __restrict__ d32) {
    constexpr int W = 2 * P + 1, S = W * W;
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I >= (long long)n * n) return;
    int j = (int)(I / n), i = (int)(I - (long long)j * n);
    int ci = i % (P + 1), cj = j % (P + 1);
    int c = ci + (P + 1) * cj;
    int ni = (n - ci + P) / (P + 1);
    int k = i / (P + 1) + ni * (j / (P + 1));
    double v = c64[((size_t)c * S + (P + W * P)) * ncp + k];
    d64[I] = v;
    d32[I] = (float)v;
}

// out = a - b (elementwise)
__global__ void __launch_bounds__(kBlock) k_sub(const double* __restrict__ a,
                                                const double* __restrict__ b,
                                                double* __restrict__ out, long long N) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I < N) out[I] = a[I] - b[I];
}

// Gather selected FP64 rows of a colour-blocked stencil into natural form.
template <int P>
__global__ void k_gather_rows(const double* __restrict__ c64, int n, int ncp,
                              const long long* __restrict__ rows, int nrows,
                              double* __restrict__ out) {
    constexpr int W = 2 * P + 1, S = W * W;
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= nrows * S) return;
    int r = t / S, o = t - r * S;
    long long I = rows[r];
    int j = (int)(I / n), i = (int)(I - (long long)j * n);
    int ci = i % (P + 1), cj = j % (P + 1);
    int c = ci + (P + 1) * cj;
    int ni = (n - ci + P) / (P + 1);
    int k = i / (P + 1) + ni * (j / (P + 1));
    out[t] = c64[((size_t)c * S + o) * ncp + k];
}

}  // namespace igamg
