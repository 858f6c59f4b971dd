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

// Ordering point between two colour steps.  Several waves: a workgroup
// barrier.  One wave (kSolo: the values a step reads were written by the same
// wave): its LDS operations run in issue order, so waiting for its own
// outstanding LDS operations, with the compiler kept from moving memory
// accesses across the point, orders the updates without a workgroup barrier.
template <bool kSolo>
__device__ __forceinline__ void pf_sync() {
    if constexpr (kSolo)
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    else
        __syncthreads();
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
    return __builtin_nontemporal_load(p);
}

// Pointers that kernels read from memory (argument tables of batched launches)
// are generic; these casts state that they address global memory, so that the
// loads are global (vmcnt) rather than flat (which an LDS wait also waits for).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
    return (__attribute__((address_space(1))) T*)p;
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

// Zero values kept before and after every FP32 iterate vector (at least p).
constexpr int kXPad = 64;

typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

// W consecutive floats from a 4-byte aligned address with 16/8/4-byte loads.
template <int W>
__device__ __forceinline__ void load_window(const float* p, float (&v)[W]) {
#pragma unroll
    for (int m = 0; m + 4 <= W; m += 4) {
        const f4u q = *reinterpret_cast<const f4u*>(p + m);
        v[m] = q[0];
        v[m + 1] = q[1];
        v[m + 2] = q[2];
        v[m + 3] = q[3];
    }
    constexpr int m = W - W % 4;
    if constexpr (W % 4 >= 2) {
        const f2u q = *reinterpret_cast<const f2u*>(p + m);
        v[m] = q[0];
        v[m + 1] = q[1];
    }
    if constexpr (W % 2 == 1) v[W - 1] = p[W - 1];
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
    static constexpr int kP = P, W = 2 * P + 1, S = W * W, NC = (P + 1) * (P + 1);
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
    // kStream: non-temporal coefficient loads (a pass that reads them once);
    // the single-workgroup cycle re-reads them and keeps them cached.
    // FP32 iterates are the library's own vectors, allocated with kXPad zero
    // values before and after: a stencil row's W values are then read from
    // column i - p with vector loads, unclamped (entries outside the row meet
    // zero coefficients).  FP64 iterates may be the caller's: clamped reads.
    template <bool kStream = true>
    __device__ __forceinline__ T slice(const T* __restrict__ x, const Pt& pt, int c, int k, int w,
                                       T& diag) const {
        const int bb = w - P;
        const T* cf = coef + ((size_t)c * S + (size_t)W * w) * ncp + k;
        const T* xr = x + (size_t)clampi(pt.j + bb, 0, n - 1) * n;
        T cv[W], xv[W];
#pragma unroll
        for (int a = 0; a < W; ++a) cv[a] = kStream ? stream_load(cf + (size_t)a * ncp) : cf[(size_t)a * ncp];
        if constexpr (std::is_same<T, float>::value)
            load_window<W>(xr + pt.i - P, xv);
        else
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
    static constexpr int kP = P, W = 2 * P + 1, NC = (P + 1) * (P + 1);
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
    // The i-row of both 1D bands (the same for every slice of a point).
    struct Bands {
        T ki[W], mi[W];
    };
    __device__ __forceinline__ void bands(const Pt& pt, Bands& B) const {
#pragma unroll
        for (int a = 0; a < W; ++a) {
            B.ki[a] = K[(size_t)pt.i * W + a];
            B.mi[a] = M[(size_t)pt.i * W + a];
        }
    }
    // Row bb = w - P of the sum-factorised product: M_jb (K_i . x_row) + K_jb (M_i . x_row).
    template <bool kStream = true>
    __device__ __forceinline__ T slice(const T* __restrict__ x, const Pt& pt, int, int, int w,
                                       T& diag) const {
        Bands B;
        bands(pt, B);
        return slice_b(B, x, pt, w, diag);
    }
    __device__ __forceinline__ T slice_b(const Bands& B, const T* __restrict__ x, const Pt& pt, int w,
                                         T& diag) const {
        const int bb = w - P;
        const T* xr = x + (size_t)clampi(pt.j + bb, 0, n - 1) * n;
        const T *ki = B.ki, *mi = B.mi;
        T xv[W];
        // FP32 iterates are padded (see Stencil2D::slice); band entries of
        // out-of-range columns are zero
        if constexpr (std::is_same<T, float>::value)
            load_window<W>(xr + pt.i - P, xv);
        else
#pragma unroll
            for (int a = 0; a < W; ++a) xv[a] = xr[clampi(pt.i + a - P, 0, n - 1)];
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
    static constexpr int kP = P, W = 2 * P + 1, NC = (P + 1) * (P + 1) * (P + 1);
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
    // The i- and j-rows of both 1D bands (the same for every slice of a point).
    struct Bands {
        T ki[W], mi[W], kj[W], mj[W];
    };
    __device__ __forceinline__ void bands(const Pt& pt, Bands& B) const {
#pragma unroll
        for (int a = 0; a < W; ++a) {
            B.ki[a] = K[(size_t)pt.i * W + a];
            B.mi[a] = M[(size_t)pt.i * W + a];
            B.kj[a] = K[(size_t)pt.j * W + a];
            B.mj[a] = M[(size_t)pt.j * W + a];
        }
    }
    // Plane cc = w - P: M_kc (sum_b M_jb Kx + K_jb Mx) + K_kc (sum_b M_jb Mx).
    template <bool kStream = true>
    __device__ __forceinline__ T slice(const T* __restrict__ x, const Pt& pt, int, int, int w,
                                       T& diag) const {
        Bands B;
        bands(pt, B);
        return slice_b(B, x, pt, w, diag);
    }
    __device__ __forceinline__ T slice_b(const Bands& B, const T* __restrict__ x, const Pt& pt, int w,
                                         T& diag) const {
        const int cc = w - P;
        const T *ki = B.ki, *mi = B.mi, *kj = B.kj, *mj = B.mj;
        const size_t nn = (size_t)n * n;
        const T* xs = x + (size_t)clampi(pt.k + cc, 0, n - 1) * nn;
        T y1 = 0, y2 = 0;
#pragma unroll
        for (int bb = -P; bb <= P; ++bb) {
            const T* xr = xs + (size_t)clampi(pt.j + bb, 0, n - 1) * n;
            T xv[W];
            if constexpr (std::is_same<T, float>::value)
                load_window<W>(xr + pt.i - P, xv);
            else
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
// kStream: non-temporal coefficient loads (levels whose coefficients do not
// stay in cache between the passes of a sweep); cached loads otherwise.
template <class Op, bool kStream = true>
__device__ __forceinline__ void gs_colour_body(const Op& A, const typename Op::T* __restrict__ b,
                                               typename Op::T* __restrict__ x, int c, int blk) {
    using T = typename Op::T;
    __shared__ T part[Op::NW][64];
    __shared__ T dg[64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int k = blk * 64 + lane;
    typename Op::Pt pt;
    bool ok = A.point(c, k, pt);
    // the finishing wave loads x_I and b_I together with its slice (no other
    // thread writes them in this pass), keeping one memory latency per pass
    T xo = 0, bo = 0;
    if (w == 0 && ok) {
        xo = x[pt.I];
        bo = b[pt.I];
    }
    T d = 1, sl = 0;
    if (ok) sl = A.template slice<kStream>(x, pt, c, k, w, d);
    part[w][lane] = sl;
    if (w == Op::NW / 2) dg[lane] = d;
    __syncthreads();
    if (w == 0 && ok) {
        T acc = 0;
#pragma unroll
        for (int v = 0; v < Op::NW; ++v) acc += part[v][lane];
        x[pt.I] = xo + (bo - acc) / dg[lane];
    }
}

template <class Op, bool kStream = true>
__global__ void __launch_bounds__(64 * Op::NW) k_gs_colour_sliced(Op A,
                                                                  const typename Op::T* __restrict__ b,
                                                                  typename Op::T* __restrict__ x,
                                                                  int c) {
    gs_colour_body<Op, kStream>(A, b, x, c, xcd_swizzle(blockIdx.x, gridDim.x));
}

// ---- row-class multicolour Gauss-Seidel (stored 2D stencils) ---------------
//
// The colours (ci, r), ci = 0..p, of one row class r are the points of the
// rows j = r (mod p+1).  Rows of one class lie p+1 apart, beyond the stencil's
// reach, so colour (ci, r) meets the values updated earlier in the class only
// along its own row, and no row that it reads from another class is written
// while the class is swept.  One workgroup per row of the class therefore runs
// the p+1 colour steps in order, separated by workgroup barriers, with the
// iterates of rows j-p..j+p staged in LDS: the result is that of p+1 separate
// colour passes (same products and sums in the same order), in one launch.
//
// One lane per point keeps every coefficient load a contiguous 64-value
// segment.  The coefficients of the next kRowDepth colour steps are loaded
// ahead into a ring of register sets and stay in flight across the LDS-only
// barriers, as far as the register file allows.

constexpr int kRowThreads = 512;
constexpr int kRowPadL = 8;          // zero columns left of column 0 (>= p)
constexpr int kRowMaxStride = 1056;  // LDS row stride limit: n <= kRowMaxStride - 2 kRowPadL

__host__ __device__ constexpr int row_stride(int n) { return (n + 2 * kRowPadL + 3) & ~3; }
__host__ __device__ constexpr int row_max_n() { return kRowMaxStride - 2 * kRowPadL; }
__host__ __device__ constexpr int row_points(int p, int n) { return (n + p) / (p + 1); }
// One point of every colour step per lane, in one workgroup.
__host__ __device__ constexpr bool row_fits(int p, int n) {
    return n <= row_max_n() && row_points(p, n) <= kRowThreads;
}
__host__ __device__ constexpr int row_threads(int p, int n) { return ((row_points(p, n) + 63) / 64) * 64; }

template <class Op>
struct RowRegs {
    typename Op::T cv[Op::S];
    typename Op::T bv;
};
// One colour step's coefficients per lane (S + 1 values) must fit the register
// budget of 512 threads: FP64 up to p = 4, FP32 up to p = 5.  (At p = 5 no
// step can be loaded ahead; on the finest 1024^2 level the row-class launches
// are then no faster than one launch per colour, on the coarser, launch-bound
// levels they are: the autotuner chooses per level.)
template <class Op>
constexpr bool row_kernel_ok() {
    return (Op::S + 1) * (int)sizeof(typename Op::T) / 4 <= 170;
}
// Colour steps loaded ahead of the one being updated (register budget of the
// ring: about half of the 256 registers a lane has at 512 threads).
// Measured on the 1024^2 annulus: FP32 at p = 4 gains from one step ahead
// (21.9 against 22.8 us per finest launch, 205 registers) although its ring
// exceeds the budget; two steps ahead at p = 3 (191 registers) lose (18.6
// against 17.3 us).
template <class Op>
constexpr int row_depth() {
    constexpr int per = (Op::S + 1) * (int)sizeof(typename Op::T) / 4;
    constexpr int d = (Op::kP == 4 && sizeof(typename Op::T) == 4) ? 1 : 120 / per - 1;
    return d < 0 ? 0 : (d > Op::kP ? Op::kP : d);
}

// Loads of colour step s for point ii of the row: unconditional (threads past
// the colour's points load a valid entry they do not use), so each wait
// counts only the loads issued before it.  32-bit byte offsets from the
// uniform coefficient base (the host keeps a level's coefficients below
// 4 GiB) need one register per load in flight.
template <class Op, bool kStream>
__device__ __forceinline__ void row_fetch(const Op& A, const typename Op::T* bj, int r, int jj, int s, int ii,
                                          RowRegs<Op>& q) {
    using T = typename Op::T;
    constexpr int P = Op::kP, S = Op::S;
    const int n = A.n, ni = (n - s + P) / (P + 1);
    const int iic = min(ii, max(ni - 1, 0));
    const int c = s + (P + 1) * r;
    const char* base = (const char*)A.coef;
    const unsigned pt_off = (unsigned)(((size_t)c * S * A.ncp + (size_t)ni * jj + iic) * sizeof(T));
    const unsigned col = (unsigned)(A.ncp * sizeof(T));
#pragma unroll
    for (int o = 0; o < S; ++o) {
        const T* ptr = (const T*)(base + (pt_off + (unsigned)o * col));
        q.cv[o] = kStream ? stream_load(ptr) : *ptr;
    }
    q.bv = bj[min(s + (P + 1) * iic, n - 1)];
}

// Gauss-Seidel update of point ii of colour step s of the staged row.
template <class Op>
__device__ __forceinline__ void row_update(const typename Op::T* xs, typename Op::T* xrow, int RS, int s,
                                           int ii, int ni, const RowRegs<Op>& q) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W;
    if (ii >= ni) return;
    const int i = s + (P + 1) * ii;
    T acc = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const T* xr = xs + w * RS + kRowPadL + i - P;
        T sl = 0;
#pragma unroll
        for (int a = 0; a < W; ++a) sl = fma(q.cv[w * W + a], xr[a], sl);
        acc += sl;
    }
    xrow[i] = xrow[i] + (q.bv - acc) / q.cv[P * W + P];
}

// Rows j-P..j+P of x into the LDS row store (zero outside the grid and in
// the pads), kRowStageBatch values per thread at a time: the loads of a
// batch are issued together (clamped addresses), then stored.
constexpr int kRowStageBatch = 8;
template <typename T, int P>
__device__ __forceinline__ void row_stage(const T* __restrict__ x, int n, int j, int RS, T* xs) {
    constexpr int W = 2 * P + 1;
    const int total = W * RS, bd = blockDim.x;
    for (int e0 = threadIdx.x; e0 < total; e0 += kRowStageBatch * bd) {
        T v[kRowStageBatch];
        bool ok[kRowStageBatch];
#pragma unroll
        for (int k = 0; k < kRowStageBatch; ++k) {
            const int e = min(e0 + k * bd, total - 1);
            const int w = e / RS, i = e - w * RS - kRowPadL, jr = j + w - P;
            ok[k] = jr >= 0 && jr < n && i >= 0 && i < n;
            const unsigned off = (unsigned)(clampi(jr, 0, n - 1) * n + clampi(i, 0, n - 1)) * (unsigned)sizeof(T);
            v[k] = *(const T*)((const char*)x + off);
        }
#pragma unroll
        for (int k = 0; k < kRowStageBatch; ++k) {
            const int e = e0 + k * bd;
            if (e < total) xs[e] = ok[k] ? v[k] : (T)0;
        }
    }
}

// Row jj of class r (one workgroup; at least row_threads(p, n) threads).
template <class Op, bool kStream>
__device__ __forceinline__ void rowclass_body(const Op& A, const typename Op::T* __restrict__ b,
                                              typename Op::T* __restrict__ x, int r, int jj) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W, D = row_depth<Op>();
    __shared__ __align__(16) T xs[W * kRowMaxStride];
    const int n = A.n, RS = row_stride(n);
    const int j = r + (P + 1) * jj;
    const T* bj = b + (size_t)j * n;
    const int t = threadIdx.x;
    RowRegs<Op> q[D + 1];
#pragma unroll
    for (int s = 0; s <= D; ++s) row_fetch<Op, kStream>(A, bj, r, jj, s, t, q[s]);
    row_stage<T, P>(x, n, j, RS, xs);
    __syncthreads();
    T* xrow = xs + P * RS + kRowPadL;
#pragma unroll
    for (int s = 0; s <= P; ++s) {
        const int ni = (n - s + P) / (P + 1);
        row_update<Op>(xs, xrow, RS, s, t, ni, q[s % (D + 1)]);
        if (s + D + 1 <= P) row_fetch<Op, kStream>(A, bj, r, jj, s + D + 1, t, q[s % (D + 1)]);
        __syncthreads();
    }
    T* xj = x + (size_t)j * n;
    for (int i = t; i < n; i += blockDim.x) xj[i] = xrow[i];
}

template <class Op, bool kStream = true>
__global__ void __launch_bounds__(kRowThreads) k_gs_rowclass(Op A, const typename Op::T* __restrict__ b,
                                                             typename Op::T* __restrict__ x, int r) {
    rowclass_body<Op, kStream>(A, b, x, r, xcd_swizzle(blockIdx.x, gridDim.x));
}

// ---- row-class multicolour Gauss-Seidel (sum-factorised operators) ----------
//
// The colours of one row class are the points of the x-rows with j = cj (2D)
// or with j = cj and k = ck (3D, mod p+1); the class's p+1 colours ci differ
// only along the row.  Two rows of a class lie p+1 or more apart in j or in k,
// beyond the operator's reach, so one workgroup per row runs the class's p+1
// colour steps in order, and no row that it reads from another class is
// written meanwhile.  Classes run in colour order, so a sweep is the
// multicolour sweep of the per-colour kernel (the same updates in the same
// order; the products are summed in another order).
// With A = K(x)M(x)M + M(x)K(x)M + M(x)M(x)K (3D; K(x)M + M(x)K in 2D; x index
// fastest), the product at (i, j, k) factors through contractions over the
// y (and z) bands:
//   (A x)_i = sum_a Kx_{i,a} u_{i+a} + Mx_{i,a} v_{i+a},
//   3D: u_{i'} = sum_{b,c} My_{j,b} Mz_{k,c} x_{i', j+b, k+c},
//       v_{i'} = sum_{b,c} (Ky_{j,b} Mz_{k,c} + My_{j,b} Kz_{k,c}) x_{i', j+b, k+c};
//   2D: u_{i'} = sum_b My_{j,b} x_{i', j+b},  v_{i'} = sum_b Ky_{j,b} x_{i', j+b}.
// The term of the row itself (b = c = 0) is split off: the rest comes from the
// neighbouring rows, which the class does not write, and is computed once per
// row; the colour steps are then 1D Gauss-Seidel steps along the row with the
// in-row coupling m00 Kx + g00 Mx (3D: m00 = My_{j,0} Mz_{k,0}, g00 = Ky_{j,0}
// Mz_{k,0} + My_{j,0} Kz_{k,0}; 2D: m00 = My_{j,0}, g00 = Ky_{j,0}).  Per
// point and sweep in 3D: (2p+1)^2 - 1 loads and about 2 (2p+1)^2 FMAs, against
// (2p+1)^3 of each per colour pass.

constexpr int kRowKronThreads = 1024;
constexpr int kRowKronMaxN = kRowKronThreads;  // one lane per point of the row

template <class Op>
constexpr bool is_kron3() {
    return std::is_same<typename Op::Pt, Pt3>::value;
}

// Offset of the row (j, k) in x (k ignored in 2D).
template <class Op>
__device__ __forceinline__ size_t kron_row_offset(int n, int j, int k) {
    if constexpr (is_kron3<Op>())
        return ((size_t)k * n + j) * n;
    else
        return (size_t)j * n;
}

// u, v of column i of the row (j, k); without the row's own term unless kSelf.
// Neighbour rows outside the grid have zero band entries: their addresses are
// clamped and the loads stay unconditional.  kAhead: every load issued before
// the first product (x in memory); else plane by plane (x in LDS, where the
// registers of 48 values in flight cost more than the latency they hide).
template <class Op, bool kSelf, bool kAhead = true>
__device__ __forceinline__ void kron_row_contract(const Op& A, const typename Op::T* __restrict__ x, int j,
                                                  int k, int i, typename Op::T& u, typename Op::T& v) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W, WA = kAhead ? W : 1;
    const int n = A.n;
    if constexpr (!is_kron3<Op>()) {
        T xv[W];
#pragma unroll
        for (int b = 0; b < W; ++b)
            xv[b] = (!kSelf && b == P) ? (T)0 : x[(size_t)clampi(j + b - P, 0, n - 1) * n + i];
        u = 0;
        v = 0;
#pragma unroll
        for (int b = 0; b < W; ++b) {
            if (!kSelf && b == P) continue;
            u = fma(A.M[(size_t)j * W + b], xv[b], u);
            v = fma(A.K[(size_t)j * W + b], xv[b], v);
        }
        return;
    } else {
        const size_t nn = (size_t)n * n;
        T xv[WA][W];
        auto load_plane = [&](int c, T (&q)[W]) {
            const T* xs = x + (size_t)clampi(k + c - P, 0, n - 1) * nn + i;
#pragma unroll
            for (int b = 0; b < W; ++b)
                q[b] = (!kSelf && b == P && c == P) ? (T)0 : xs[(size_t)clampi(j + b - P, 0, n - 1) * n];
        };
        if constexpr (kAhead) {
#pragma unroll
            for (int c = 0; c < W; ++c) load_plane(c, xv[c]);
        }
        u = 0;
        v = 0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            T(&q)[W] = xv[kAhead ? c : 0];
            if constexpr (!kAhead) load_plane(c, q);
            T sm = 0, sk = 0;
#pragma unroll
            for (int b = 0; b < W; ++b) {
                if (!kSelf && b == P && c == P) continue;
                sm = fma(A.M[(size_t)j * W + b], q[b], sm);
                sk = fma(A.K[(size_t)j * W + b], q[b], sk);
            }
            const T mz = A.M[(size_t)k * W + c], kz = A.K[(size_t)k * W + c];
            u = fma(mz, sm, u);
            v = fma(kz, sm, fma(mz, sk, v));
        }
    }
}

// The row's own coupling factors: the coefficient of x_{i+a} in its own row is
// m00 Kx_{i,a} + g00 Mx_{i,a}.
template <class Op>
__device__ __forceinline__ void kron_row_self(const Op& A, int j, int k, typename Op::T& m00,
                                              typename Op::T& g00) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W;
    const T mj = A.M[(size_t)j * W + P], kj = A.K[(size_t)j * W + P];
    if constexpr (is_kron3<Op>()) {
        const T mk = A.M[(size_t)k * W + P], kk = A.K[(size_t)k * W + P];
        m00 = mj * mk;
        g00 = fma(kj, mk, mj * kk);
    } else {
        m00 = mj;
        g00 = kj;
    }
}

// LDS bytes of the row kernels: u, v (and the row's iterate) with p zeros on
// either side.
__host__ __device__ constexpr int row_kron_lds_bytes(int p, int n, int arrays, int elem) {
    return arrays * (n + 2 * p) * elem;
}

template <class Op>
__global__ void __launch_bounds__(kRowKronThreads) k_gs_rowclass_kron(Op A, const typename Op::T* __restrict__ b,
                                                                      typename Op::T* __restrict__ x, int cj,
                                                                      int ck) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W;
    extern __shared__ __align__(16) unsigned char row_kron_lds[];
    const int n = A.n, L = n + 2 * P;
    T* su = (T*)row_kron_lds;
    T* sv = su + L;
    T* sx = sv + L;
    const int nj = (n - cj + P) / (P + 1);
    const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
    const int kq = blk / nj, jq = blk - kq * nj;
    const int j = cj + (P + 1) * jq, k = ck + (P + 1) * kq;
    const int t = threadIdx.x, i = min(t, n - 1);
    const size_t row = kron_row_offset<Op>(n, j, k);
    const T xo = x[row + i], bo = b[row + i];
    T kx[W], mx[W];
#pragma unroll
    for (int a = 0; a < W; ++a) {
        kx[a] = A.K[(size_t)i * W + a];
        mx[a] = A.M[(size_t)i * W + a];
    }
    T u, v;
    kron_row_contract<Op, false>(A, x, j, k, i, u, v);
    if (t < n) {
        su[t + P] = u;
        sv[t + P] = v;
        sx[t + P] = xo;
    }
    if (t < P) {  // pads (threads t < P exist for every n; threads past n need not)
        su[t] = 0;
        sv[t] = 0;
        sx[t] = 0;
        su[n + P + t] = 0;
        sv[n + P + t] = 0;
        sx[n + P + t] = 0;
    }
    __syncthreads();
    T m00, g00;
    kron_row_self(A, j, k, m00, g00);
    T rest = 0, cr[W];
#pragma unroll
    for (int a = 0; a < W; ++a) {
        if (t < n) {
            rest = fma(kx[a], su[t + a], rest);
            rest = fma(mx[a], sv[t + a], rest);
        }
        cr[a] = fma(m00, kx[a], g00 * mx[a]);
    }
    const int s_own = t % (P + 1);
#pragma unroll
    for (int s = 0; s <= P; ++s) {
        if (t < n && s_own == s) {
            T acc = rest;
#pragma unroll
            for (int a = 0; a < W; ++a) acc = fma(cr[a], sx[t + a], acc);
            sx[t + P] = sx[t + P] + (bo - acc) / cr[P];
        }
        if (s < P) __syncthreads();
    }
    if (t < n) x[row + t] = sx[t + P];
}

// ---- plane-class multicolour Gauss-Seidel (sum-factorised 3D operators) ----
//
// One launch per plane class ck: the planes k = ck (mod p+1) lie p+1 apart,
// so one workgroup per plane sweeps the plane's (p+1)^2 colours (ci, cj, ck)
// in colour order.  The workgroup first copies into LDS, in one bulk load,
// the 2p+1 planes k-p..k+p (the other planes do not change during the
// launch; its own plane is updated there), the plane of b and the 1D bands;
// then it runs the row classes cj one after the other (a workgroup barrier
// each), the p+1 colour steps of a row by one wave (ordered by the wave's own
// LDS operations), with no memory access but LDS until the plane is written
// back.  The contraction and the summation order are those of
// k_gs_rowclass_kron, so the iterates are the same, from p+1 launches per
// sweep instead of (p+1)^2.  Levels of up to 64 unknowns per direction (one
// lane per point of a row) whose planes fit the LDS: on larger levels the
// planes of a class are too few workgroups to fill the GPU (a variant with
// two points per lane at 65^3 took twice the time of the row-class launches).
constexpr int kPlane3MaxN = 64;
constexpr int kPlane3MaxLds = 160 * 1024;  // LDS per workgroup (dynamic; the launch attribute is raised)
// Waves per workgroup: one per row of a class, at most 16.
__host__ __device__ constexpr int plane3_waves(int p, int n) {
    return (n + p) / (p + 1) < 16 ? (n + p) / (p + 1) : 16;
}
// LDS: 2p+1 planes of x, the plane of b, the K and M bands, and each wave's
// two padded rows of partial sums.
__host__ __device__ constexpr long long plane3_lds_bytes(int p, int n, int elem) {
    return ((long long)(2 * p + 2) * n * n + 2LL * n * (2 * p + 1) + 2LL * plane3_waves(p, n) * (n + 2 * p)) *
           elem;
}

// kron_row_contract<Op, false> (3D) with the planes k-p..k+p read from the
// LDS slab (plane c at slab + c n^2) and the bands from LDS.
template <class Op>
__device__ __forceinline__ void plane3_contract(const typename Op::T* sK, const typename Op::T* sM,
                                                const typename Op::T* slab, int n, int j, int k, int i,
                                                typename Op::T& u, typename Op::T& v) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W;
    const int nn = n * n;
    u = 0;
    v = 0;
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const T* xs = slab + c * nn + i;
        T xv[W];
#pragma unroll
        for (int b = 0; b < W; ++b) xv[b] = (b == P && c == P) ? (T)0 : xs[clampi(j + b - P, 0, n - 1) * n];
        T sm = 0, sk = 0;
#pragma unroll
        for (int b = 0; b < W; ++b) {
            if (b == P && c == P) continue;
            sm = fma(sM[j * W + b], xv[b], sm);
            sk = fma(sK[j * W + b], xv[b], sk);
        }
        const T mz = sM[k * W + c], kz = sK[k * W + c];
        u = fma(mz, sm, u);
        v = fma(kz, sm, fma(mz, sk, v));
    }
}

template <class Op>
__global__ void __launch_bounds__(1024) k_gs_planeclass3(Op A, const typename Op::T* __restrict__ b,
                                                         typename Op::T* __restrict__ x, int ck) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W;
    extern __shared__ __align__(16) unsigned char row_kron_lds[];
    const int n = A.n, L = n + 2 * P, nwave = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63,
              i = min(lane, n - 1);
    const int nn = n * n;
    T* slab = (T*)row_kron_lds;
    T* sb = slab + W * nn;
    T* sK = sb + nn;
    T* sM = sK + n * W;
    T* su = sM + n * W + wave * 2 * L;
    T* sv = su + L;
    const int k = ck + (P + 1) * xcd_swizzle(blockIdx.x, gridDim.x);
    // planes k-p..k+p (clamped to the grid: their band entries are zero) and
    // b, the 2p+2 loads of a point in flight before their stores; the bands
    {
        const T* src[W + 1];
#pragma unroll
        for (int c = 0; c < W; ++c) src[c] = x + (size_t)clampi(k + c - P, 0, n - 1) * nn;
        src[W] = b + (size_t)k * nn;
        for (int e = threadIdx.x; e < nn; e += blockDim.x) {
            T r[W + 1];
#pragma unroll
            for (int c = 0; c <= W; ++c) r[c] = src[c][e];
#pragma unroll
            for (int c = 0; c <= W; ++c) slab[c * nn + e] = r[c];
        }
        for (int e = threadIdx.x; e < n * W; e += blockDim.x) {
            sK[e] = A.K[e];
            sM[e] = A.M[e];
        }
    }
    if (lane < P) {
        su[lane] = 0;
        sv[lane] = 0;
        su[n + P + lane] = 0;
        sv[n + P + lane] = 0;
    }
    __syncthreads();
    T* xp = slab + P * nn;  // the plane itself
    const T mk = sM[k * W + P], kk = sK[k * W + P];
    const int s_own = lane % (P + 1);
    for (int cj = 0; cj <= P; ++cj) {
        const int nj = (n - cj + P) / (P + 1);
        for (int jq = wave; jq < nj; jq += nwave) {
            const int j = cj + (P + 1) * jq;
            T* xr = xp + j * n;
            T u, v;
            plane3_contract<Op>(sK, sM, slab, n, j, k, i, u, v);
            if (lane < n) {
                su[lane + P] = u;
                sv[lane + P] = v;
            }
            pf_sync<true>();
            const T mj = sM[j * W + P], kj = sK[j * W + P];
            const T m00 = mj * mk, g00 = fma(kj, mk, mj * kk);
            const T bo = sb[j * n + i];
            T rest = 0, cr[W];
#pragma unroll
            for (int a = 0; a < W; ++a) {
                const T kx = sK[i * W + a], mx = sM[i * W + a];
                rest = fma(kx, su[i + a], rest);
                rest = fma(mx, sv[i + a], rest);
                cr[a] = fma(m00, kx, g00 * mx);
            }
#pragma unroll
            for (int s = 0; s <= P; ++s) {
                if (lane < n && s_own == s) {
                    T acc = rest;
#pragma unroll
                    for (int a = 0; a < W; ++a) acc = fma(cr[a], xr[clampi(lane + a - P, 0, n - 1)], acc);
                    xr[lane] = xr[lane] + (bo - acc) / cr[P];
                }
                pf_sync<true>();
            }
        }
        __syncthreads();
    }
    T* xg = x + (size_t)k * nn;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) xg[e] = xp[e];
}

// Residual-type products of a sum-factorised operator, one workgroup per
// x-row (natural order): r = b - A x (mode 0), y = A x (mode 1), damped
// Jacobi step (mode 2); optionally the row's sum of squares of the output in
// partial[row] (fixed reduction order).
template <class Op, typename Tout>
__global__ void __launch_bounds__(kRowKronThreads) k_residual_row_kron(Op A, const typename Op::T* __restrict__ b,
                                                                       const typename Op::T* __restrict__ x,
                                                                       Tout* __restrict__ out, int mode,
                                                                       double omega, double* __restrict__ partial) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W;
    extern __shared__ __align__(16) unsigned char row_kron_lds[];
    __shared__ double red[kRowKronThreads / 64];
    const int n = A.n, L = n + 2 * P;
    T* su = (T*)row_kron_lds;
    T* sv = su + L;
    const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
    const int k = is_kron3<Op>() ? blk / n : 0, j = blk - k * n;
    const int t = threadIdx.x, i = min(t, n - 1);
    const size_t row = kron_row_offset<Op>(n, j, k);
    T bo = 0, xo = 0;
    if (mode != 1) bo = b[row + i];
    if (mode == 2) xo = x[row + i];
    T kx[W], mx[W];
#pragma unroll
    for (int a = 0; a < W; ++a) {
        kx[a] = A.K[(size_t)i * W + a];
        mx[a] = A.M[(size_t)i * W + a];
    }
    T u, v;
    kron_row_contract<Op, true>(A, x, j, k, i, u, v);
    if (t < n) {
        su[t + P] = u;
        sv[t + P] = v;
    }
    if (t < P) {  // pads
        su[t] = 0;
        sv[t] = 0;
        su[n + P + t] = 0;
        sv[n + P + t] = 0;
    }
    __syncthreads();
    double sq = 0.0;
    if (t < n) {
        T acc = 0;
#pragma unroll
        for (int a = 0; a < W; ++a) {
            acc = fma(kx[a], su[t + a], acc);
            acc = fma(mx[a], sv[t + a], acc);
        }
        T r;
        if (mode == 0)
            r = bo - acc;
        else if (mode == 1)
            r = acc;
        else {
            T m00, g00;
            kron_row_self(A, j, k, m00, g00);
            const T d = fma(m00, kx[P], g00 * mx[P]);
            r = xo + (T)omega * (bo - acc) / d;
        }
        out[row + t] = (Tout)r;
        sq = (double)r * (double)r;
    }
    if (partial) {
        const double tot = block_sum(sq, red);
        if (t == 0) partial[blk] = tot;
    }
}

// The same products on the large 3D levels, one workgroup per x-row j and
// run of kResRollPlanes planes k.  The y-contractions of a plane (the sums
// over b of M[j,b] x and K[j,b] x along the row's 2p+1 neighbour rows) enter
// the 2p+1 output planes around it; they are kept in a window of registers as
// k advances, so that each x value is read from L2 about (2p+1)(1 + 2p/8)
// times rather than (2p+1)^2.  The loads of the next two planes are in flight
// during the current plane's output: the 1D bands sit in LDS, and b of the
// next output plane is requested before the prefetched planes, so that no
// wait for a value in use (vector memory counts drain in issue order) waits
// for the prefetch.  Every
// sum is formed in the order of k_residual_row_kron (so the outputs and the
// per-row sums of squares in partial[k n + j] are the same, bit for bit).  On
// levels below kResRollMinN unknowns per direction the chain of planes of a
// workgroup outlasts the whole per-row launch, which is used there (and above
// kResRollMaxN, rows of more than 512 threads).
constexpr int kResRollPlanes = 8;
constexpr int kResRollMinN = 96;
constexpr int kResRollMaxN = 512;
// LDS: the squares of the run's outputs (one per plane and thread) and their
// per-wave sums (FP64), the 1D bands and the two (u, v) row buffers.
__host__ __device__ constexpr int res_roll_lds_bytes(int p, int n, int elem) {
    return kResRollPlanes * (((n + 63) / 64) * 64 + kResRollMaxN / 64) * 8 +
           (2 * n * (2 * p + 1) + 4 * (n + 2 * p)) * elem;
}
template <class Op, typename Tout>
__global__ void __launch_bounds__(kResRollMaxN) k_residual_roll_kron3(Op A, const typename Op::T* __restrict__ b,
                                                                      const typename Op::T* __restrict__ x,
                                                                      Tout* __restrict__ out, int mode, double omega,
                                                                      double* __restrict__ partial) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W;
    static_assert(is_kron3<Op>(), "3D sum-factorised operators");
    extern __shared__ __align__(16) unsigned char row_kron_lds[];
    constexpr int KC = kResRollPlanes, MW = kResRollMaxN / 64;
    const int n = A.n, L = n + 2 * P;
    const size_t nn = (size_t)n * n;
    double* sqb = (double*)row_kron_lds;  // KC x blockDim squares
    double* redk = sqb + KC * blockDim.x;  // KC x MW per-wave sums
    T* cK = (T*)(redk + KC * MW);          // the 1D bands, n x (2p+1) each
    T* cM = cK + n * W;
    T* sbuf = cM + n * W;  // two buffers of (u row, v row), each padded by p zeros
    const int lb = xcd_swizzle(blockIdx.x, gridDim.x);
    const int kc = lb / n, j = lb - kc * n;
    const int k0 = kc * kResRollPlanes, k1 = min(k0 + kResRollPlanes, n);
    const int t = threadIdx.x, i = min(t, n - 1);
    // x at (plane q clamped, rows j-p..j+p clamped, column i)
    auto load = [&](int q, T (&r)[W]) {
        const T* xs = x + (size_t)clampi(q, 0, n - 1) * nn + i;
#pragma unroll
        for (int bb = 0; bb < W; ++bb) r[bb] = xs[(size_t)clampi(j + bb - P, 0, n - 1) * n];
    };
    for (int e = t; e < n * W; e += blockDim.x) {
        cK[e] = A.K[e];
        cM[e] = A.M[e];
    }
    // Every step issues the same loads (clamped indices; b replaced by x where
    // it is not read), so that the compiler's wait for a plane counts the
    // loads issued after it on every path and leaves them in flight.
    const T* bsrc = (mode != 1) ? b : x;
    T buf0[W], buf1[W];
    load(k0 - P, buf0);
    load(k0 - P + 1, buf1);  // steps >= 2p+1 >= 3
    // b and x at the next output plane (x read by the Jacobi step only)
    T bo = bsrc[(size_t)k0 * nn + (size_t)j * n + i], xo = x[(size_t)k0 * nn + (size_t)j * n + i];
    if (t < P) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            sbuf[q * L + t] = 0;
            sbuf[q * L + n + P + t] = 0;
        }
    }
    __syncthreads();
    T sm[W], sk[W];  // y-contractions of planes k-p..k+p (index c = plane - k + p)
    const int steps = (k1 - k0) + 2 * P;
    // step st: the plane k0-p+st enters the window (from buf, which then takes
    // the loads of the plane two steps on); from st = 2p on, plane k0+st-2p out
    auto step = [&](int st, T (&buf)[W]) {
#pragma unroll
        for (int c = 0; c + 1 < W; ++c) {
            sm[c] = sm[c + 1];
            sk[c] = sk[c + 1];
        }
        {
            T a0 = 0, a1 = 0;
#pragma unroll
            for (int bb = 0; bb < W; ++bb) {
                a0 = fma(cM[j * W + bb], buf[bb], a0);
                a1 = fma(cK[j * W + bb], buf[bb], a1);
            }
            sm[W - 1] = a0;
            sk[W - 1] = a1;
        }
        const int k = k0 + st - 2 * P;
        const size_t row = (size_t)k * nn + (size_t)j * n;
        const T bk = bo, xk = xo;
        {
            const size_t nxt = (size_t)clampi(k + 1, k0, k1 - 1) * nn + (size_t)j * n + i;
            bo = bsrc[nxt];
            xo = x[nxt];
        }
        load(k0 - P + st + 2, buf);
        if (st < 2 * P) return;
        T u = 0, v = 0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const T mz = cM[k * W + c], kz = cK[k * W + c];
            u = fma(mz, sm[c], u);
            v = fma(kz, sm[c], fma(mz, sk[c], v));
        }
        T* su = sbuf + (k & 1) * 2 * L;
        T* sv = su + L;
        if (t < n) {
            su[t + P] = u;
            sv[t + P] = v;
        }
        __syncthreads();
        double sq = 0.0;
        if (t < n) {
            T acc = 0;
#pragma unroll
            for (int a = 0; a < W; ++a) {
                acc = fma(cK[i * W + a], su[t + a], acc);
                acc = fma(cM[i * W + a], sv[t + a], acc);
            }
            T r;
            if (mode == 0)
                r = bk - acc;
            else if (mode == 1)
                r = acc;
            else {
                const T mj = cM[j * W + P], kj = cK[j * W + P], mk = cM[k * W + P], kk = cK[k * W + P];
                const T m00 = mj * mk, g00 = fma(kj, mk, mj * kk);
                const T d = fma(m00, cK[i * W + P], g00 * cM[i * W + P]);
                r = xk + (T)omega * (bk - acc) / d;
            }
            out[row + t] = (Tout)r;
            sq = (double)r * (double)r;
        }
        if (partial) sqb[(k - k0) * blockDim.x + t] = sq;
    };
    int st = 0;
    for (; st + 1 < steps; st += 2) {
        step(st, buf0);
        step(st + 1, buf1);
    }
    if (st < steps) step(st, buf0);
    // The rows' sums of squares, with block_sum's tree (each wave sums its 64
    // lanes, then the wave sums in order), for all the run's planes at once.
    if (partial) {
        const int np = k1 - k0, lane = t & 63, w = t >> 6, nw = (blockDim.x + 63) >> 6;
        double v[KC];
#pragma unroll
        for (int q = 0; q < KC; ++q) v[q] = (q < np) ? sqb[q * blockDim.x + t] : 0.0;
#pragma unroll
        for (int q = 0; q < KC; ++q) v[q] = wave_sum(v[q]);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < KC; ++q) redk[q * MW + w] = v[q];
        }
        __syncthreads();
        if (t < np) {
            double tot = 0.0;
            for (int e = 0; e < nw; ++e) tot += redk[t * MW + e];
            partial[(size_t)(k0 + t) * n + j] = tot;
        }
    }
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
    T xo = 0, bo = 0;  // loaded with the slices, as in the colour pass
    if (w == 0 && ok) {
        if (mode != 1) bo = b[pt.I];
        if (mode == 2) xo = x[pt.I];
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
        if (mode == 0 || mode == 3)
            v = bo - acc;
        else if (mode == 1)
            v = acc;
        else
            v = xo + (T)omega * (bo - acc) / dg[lane];
        if (mode == 3) {  // learned-step input z = D^{-1} (b - A x) and z^2
            const float z = (float)((double)v / (double)dg[lane]);
            out[pt.I] = (Tout)z;
            sq = (double)z * z;
        } else {
            out[pt.I] = (Tout)v;
            sq = (double)v * (double)v;
        }
    }
    if (partial) {
        if (w == 0) {
            double t = wave_sum(sq);
            if (lane == 0) partial[slot] = t;
        }
    }
}

// The learned step's input when x = 0 (a level entered from a zero start):
// z = D^{-1} b and per-block sums of z^2, exactly what residual_body's mode 3
// gives for x = 0 (every product with x is +0, so b - A x = b bit for bit) over
// the same blocks, points and wave sums, but reading only b and the stencil
// centre (colour-ordered stored stencils; one wave per block).
template <class Op>
__global__ void __launch_bounds__(64) k_scaled_rhs(Op A, const typename Op::T* __restrict__ b,
                                                   float* __restrict__ out, double* __restrict__ partial) {
    using T = typename Op::T;
    static_assert(Op::kColourOrder, "colour-ordered stored stencils only");
    const int lane = threadIdx.x;
    const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
    const int bpc = A.ncp / 64;
    const int c = blk / bpc, k = (blk - c * bpc) * 64 + lane;
    typename Op::Pt pt;
    const bool ok = (c < Op::NC) && A.point(c, k, pt);
    double sq = 0.0;
    if (ok) {
        const T d = A.coef[((size_t)c * Op::S + (size_t)Op::W * Op::kP + Op::kP) * A.ncp + k];
        const float z = (float)((double)b[pt.I] / (double)d);
        out[pt.I] = z;
        sq = (double)z * z;
    }
    const double t = wave_sum(sq);
    if (lane == 0) partial[blockIdx.x] = t;
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

// Krylov kernels (flexible GMRES): per-block partial dot products of w with
// v_0 .. v_{k-1}, partial[blk * k + i]; their sums in block order; and
// w += sign * sum_i h_i v_i.
__global__ void __launch_bounds__(kBlock) k_dots_partial(const double* __restrict__ w, VecPtrs V, int k,
                                                         long long N, double* __restrict__ partial) {
    __shared__ double red[kBlock / 64];
    for (int i = 0; i < k; ++i) {
        const double* __restrict__ v = V.v[i];
        double s = 0.0;
        for (long long I = (long long)blockIdx.x * kBlock + threadIdx.x; I < N; I += (long long)gridDim.x * kBlock)
            s = fma(w[I], v[I], s);
        s = block_sum(s, red);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * k + i] = s;
    }
}

__global__ void k_dots_finalize(const double* __restrict__ partial, int nb, int k, double* __restrict__ out) {
    const int i = threadIdx.x;
    if (i >= k) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * k + i];
    out[i] = s;
}

__global__ void __launch_bounds__(kBlock) k_axpy_multi(double* __restrict__ w, VecPtrs V,
                                                       const double* __restrict__ h, int k, double sign,
                                                       long long N) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I >= N) return;
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc = fma(h[i], V.v[i][I], acc);
    w[I] += sign * acc;
}

// v = w / s (s on the host side of the call)
__global__ void __launch_bounds__(kBlock) k_scaled_copy(const double* __restrict__ w, double* __restrict__ v,
                                                        double inv, long long N) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I < N) v[I] = w[I] * inv;
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
// Window bounds of the knot-insertion transfers: a coarse B-spline of degree
// p refines into at most p + 2 fine ones (restriction window); a fine one
// receives at most floor((p + 1) / 2) + 1 coarse ones (prolongation window).
// The host checks both when it builds the tables.
__host__ __device__ constexpr int restrict_bound(int p) { return p + 2; }
__host__ __device__ constexpr int prolong_bound(int p) { return (p + 1) / 2 + 1; }

// One value of a separable 2D transfer: sum_b w_j[b] sum_a w_i[a] g(sj+b, si+a)
// over the windows of a 1D table (start st[], weights w[idx*W + a], nw rows),
// on an n x n row-major grid, indices clamped to the grid.  The windows are
// unrolled to their bound M (entries a >= W weigh zero), so all loads of a
// point are in flight together.
template <int M, typename T>
__device__ __forceinline__ T transfer2d(const T* __restrict__ g, int n, const int* __restrict__ st,
                                        const T* __restrict__ w, int W, int nw, int i, int j) {
    const int si = st[i], sj = st[j];
    const int last = nw * W - 1;
    T wi[M], wj[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const T u = w[min(i * W + a, last)], v = w[min(j * W + a, last)];
        wi[a] = (a < W) ? u : (T)0;
        wj[a] = (a < W) ? v : (T)0;
    }
    T acc = 0;
#pragma unroll
    for (int b = 0; b < M; ++b) {
        const T* row = g + (size_t)min(sj + b, n - 1) * n;
        T s = 0;
#pragma unroll
        for (int a = 0; a < M; ++a) s = fma(wi[a], row[min(si + a, n - 1)], s);
        acc = fma(wj[b], s, acc);
    }
    return acc;
}

// bc = R rf (R = P^T) and, optionally, xc = 0.
template <int P, typename T>
__global__ void __launch_bounds__(kBlock) k_restrict2d(const T* __restrict__ rf, int nf,
                                                       T* __restrict__ bc, int nc,
                                                       const int* __restrict__ rs,
                                                       const T* __restrict__ rw, int RW,
                                                       T* __restrict__ xc) {
    long long C = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (C >= (long long)nc * nc) return;
    if (xc) xc[C] = 0;
    int J = (int)(C / nc), I = (int)(C - (long long)J * nc);
    bc[C] = transfer2d<restrict_bound(P), T>(rf, nf, rs, rw, RW, nc, I, J);
}

// xf += P ec.
template <int P, typename T>
__global__ void __launch_bounds__(kBlock) k_prolong2d(const T* __restrict__ ec, int nc,
                                                      T* __restrict__ xf, int nf,
                                                      const int* __restrict__ ps,
                                                      const T* __restrict__ pw, int PW) {
    long long F = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (F >= (long long)nf * nf) return;
    int j = (int)(F / nf), i = (int)(F - (long long)j * nf);
    xf[F] += transfer2d<prolong_bound(P), T>(ec, nc, ps, pw, PW, nf, i, j);
}

// One value of a separable 3D transfer (as transfer2d, one more factor): the
// window of each plane is unrolled to M, the planes are taken in turn.
template <int M, typename T>
__device__ __forceinline__ T transfer3d(const T* __restrict__ g, int n, const int* __restrict__ st,
                                        const T* __restrict__ w, int W, int nw, int i, int j, int k) {
    const int si = st[i], sj = st[j], sk = st[k];
    const int last = nw * W - 1;
    T wi[M], wj[M], wk[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const T u = w[min(i * W + a, last)], v = w[min(j * W + a, last)], q = w[min(k * W + a, last)];
        wi[a] = (a < W) ? u : (T)0;
        wj[a] = (a < W) ? v : (T)0;
        wk[a] = (a < W) ? q : (T)0;
    }
    T acc = 0;
#pragma unroll 1
    for (int c = 0; c < M; ++c) {
        const T* sl = g + (size_t)min(sk + c, n - 1) * n * n;
        T s2 = 0;
#pragma unroll
        for (int b = 0; b < M; ++b) {
            const T* row = sl + (size_t)min(sj + b, n - 1) * n;
            T s1 = 0;
#pragma unroll
            for (int a = 0; a < M; ++a) s1 = fma(wi[a], row[min(si + a, n - 1)], s1);
            s2 = fma(wj[b], s1, s2);
        }
        acc = fma(wk[c], s2, acc);
    }
    return acc;
}

template <int P, typename T>
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
    bc[C] = transfer3d<restrict_bound(P), T>(rf, nf, rs, rw, RW, nc, I, J, K);
}

template <int P, typename T>
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
    xf[F] += transfer3d<prolong_bound(P), T>(ec, nc, ps, pw, PW, nf, i, j, k);
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
// One thread; Rg row-major ncols x ncols (global or LDS).
__device__ inline ExtrapCoeffs extrap_coefficients(const double* Rg, int ncols, int method) {
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
    c.gres = __builtin_nan("");
    c.d0 = fabs(Rg[0]);
    if (!finite) {
        c.info = -2;
        return c;
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
        return c;
    }
    double acc = 1.0;
    for (int i = 0; i < n; ++i) c.gamma[i] = d[i] / lam;
    for (int j = 0; j < q; ++j) {
        acc -= c.gamma[j];
        c.alpha[j] = acc;
    }
    // generalised residual t~ - t = sum_j gamma_j Delta s_j = Q (R gamma)
    double g2 = 0.0;
    for (int i = 0; i < n; ++i) {
        double v = 0.0;
        for (int k = i; k < n; ++k) v += R[i][k] * c.gamma[k];
        g2 += v * v;
    }
    c.gres = sqrt(g2);
    return c;
}

__global__ void k_extrap_coeffs(const double* __restrict__ Rg, int ncols, int method,
                                ExtrapCoeffs* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    *out = extrap_coefficients(Rg, ncols, method);
}

// t = s_0 + sum_{j<q} alpha_j (s_{j+1} - s_j) into out.  keep (optional)
// receives s_0, the iterate accepted before this cycle.  info -1 (no
// extrapolation): out = s_{q+1}; info -2 (non-finite coefficients): out is not
// written, so an in-place call leaves s_0 there.  `out` may alias s_0.
__global__ void __launch_bounds__(kBlock) k_extrap_combine(IterPtrs S, int q, long long N,
                                                           const ExtrapCoeffs* __restrict__ cf,
                                                           double* out, double* keep) {
    long long I = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (I >= N) return;
    int info = cf->info;
    double prev = S.s[0][I];
    if (keep) keep[I] = prev;
    if (info == -2) return;
    if (info < 0) {
        out[I] = S.s[q + 1][I];
        return;
    }
    double t = prev;
    for (int j = 0; j < q; ++j) {
        double nxt = S.s[j + 1][I];
        t = fma(cf->alpha[j], nxt - prev, t);
        prev = nxt;
    }
    out[I] = t;
}


// ---------------------------------------------------------------------------
// single-workgroup V-cycle on the small levels 0..top.  One launch replaces the
// hundreds of tiny launches those levels would need.  The iterates of all
// levels 0..top stay in LDS for the whole cycle, so a colour pass reads the
// neighbours of its points from LDS and only the read-only coefficients, b and
// r go to memory; passes are separated by workgroup barriers.

constexpr int kTailMaxLevels = 8;
constexpr int kTailThreads = 1024;
// FP32 stored stencils take the prefetching variant: the coefficients of a
// point are one 16-byte aligned record and the next colour step's records are
// in flight while the current step computes.  Two records per thread must fit
// the register budget: 512 threads (256 VGPRs) up to p = 4, 256 threads
// (512 VGPRs) for p = 5; one point per thread, so a level's colours must fit.
__host__ __device__ constexpr int pf_threads(int p) { return p <= 4 ? 512 : 256; }
template <class Op>
constexpr bool tail_prefetch() {
    if constexpr (Op::kColourOrder) return std::is_same<typename Op::T, float>::value;
    else return false;
}
// Sum-factorised 2D levels of high degree take 512 threads (256 VGPRs per
// lane), where 1024 threads' 128 spill: FP64 from p = 3, FP32 from p = 4.
template <class Op>
constexpr int tail_threads() {
    if constexpr (Op::kColourOrder)
        return tail_prefetch<Op>() ? pf_threads(Op::kP) : kTailThreads;
    else if constexpr (!std::is_same<typename Op::Pt, Pt3>::value &&
                       Op::kP >= (sizeof(typename Op::T) == 8 ? 3 : 4))
        return kTailThreads / 2;
    else
        return kTailThreads;
}
// Floats per coefficient record of degree p: (2p+1)^2 rounded up to 4.
__host__ __device__ constexpr int rec_len(int p) { return ((2 * p + 1) * (2 * p + 1) + 3) / 4 * 4; }
constexpr int kTailLdsX = 153600;    // LDS bytes for the iterates of levels 0..top
constexpr int kTailPadVals = 16;     // zero values after the last level (unclamped row reads)

// Padded LDS layout of a level's iterate for stored 2D stencils: rows
// j = -p .. n-1+p and, per row, a left pad of padl >= p columns (a multiple of
// the 128-bit vector width vw, so rows stay 16-byte aligned) and a right pad
// wide enough that the nv aligned vector reads covering a stencil row never
// leave the row.  Pads hold zeros (the coefficients of out-of-domain
// neighbours are zero as well), so no index is clamped.
__host__ __device__ constexpr int tl_vw(int bytes) { return 16 / bytes; }
__host__ __device__ constexpr int tl_padl(int p, int vw) { return ((p + vw - 1) / vw) * vw; }
__host__ __device__ constexpr int tl_nv(int p, int vw) { return (vw - 1 + 2 * p + 1 + vw - 1) / vw; }
__host__ __device__ constexpr int tl_stride(int p, int vw, int n) {
    return ((tl_padl(p, vw) + n + tl_nv(p, vw) * vw + vw - 1) / vw) * vw;
}
__host__ __device__ constexpr long long tl_size(int p, int vw, int n) {
    return (long long)(n + 2 * p) * tl_stride(p, vw, n);
}


// Unknowns of levels 0..top that fit the LDS iterate store in precision T.
template <typename T>
constexpr long long tail_capacity() {
    return kTailLdsX / (long long)sizeof(T);
}

template <class Op>
struct TailArgs {
    using T = typename Op::T;
    int top;                        // finest level handled here
    int nu1, nu2;
    int mu;                         // cycle index of Algorithm 2 (1: V-cycle, 2: W-cycle)
    int n0;                         // coarsest unknowns
    const double* Ainv;             // coarsest inverse (FP64)
    Op op[kTailMaxLevels];
    long long N[kTailMaxLevels];
    int xoff[kTailMaxLevels];       // offset of level l's iterate in the LDS store
    int boff[kTailMaxLevels];       // sum-factorised operators: offset of level l's 1D bands (K, M)
    T* x[kTailMaxLevels];           // only x[top] is read and written (in and out)
    T* b[kTailMaxLevels];
    T* r[kTailMaxLevels];
    const T* rec[kTailMaxLevels];   // per-point coefficient records (prefetching variant)
    int act[kTailMaxLevels];        // prefetching variant: waves holding points of the level's largest colour
    const int* rs[kTailMaxLevels];  // transfer tables between l-1 and l
    const T* rw[kTailMaxLevels];
    const int* ps[kTailMaxLevels];
    const T* pw[kTailMaxLevels];
    int RW[kTailMaxLevels], PW[kTailMaxLevels];
};

// Order of the steps of one mu-cycle (Algorithm 2) on levels 0..top, without
// recursion: down(l) pre-smooths level l, restricts its residual to b_{l-1}
// and zeroes x_{l-1}; coarse() solves level 0; up(l) adds the prolongated
// correction to x_l and post-smooths.  Level l calls the cycle of level l-1
// mu times on the same b_{l-1}, the later calls starting from the previous
// result.  Every thread of the workgroup runs the same sequence.
template <class Down, class Coarse, class Up>
__device__ __forceinline__ void mu_schedule(int top, int mu, Down down, Coarse coarse, Up up) {
    if (top == 0) {
        coarse();
        return;
    }
    unsigned done = 0;  // 4 bits per level: finished coarse calls of its active cycle
    int l = top;
    for (;;) {
        for (; l > 0; --l) {
            down(l);
            done &= ~(15u << (4 * l));
        }
        coarse();
        for (;;) {
            ++l;
            const unsigned d = ((done >> (4 * l)) & 15u) + 1;
            done = (done & ~(15u << (4 * l))) | (d << (4 * l));
            if ((int)d < mu) {
                --l;  // the next call of level l-1's cycle
                break;
            }
            up(l);
            if (l == top) return;
        }
    }
}

// b_c = R r_f (r_f in memory) and x_c = 0 (LDS); windows unrolled to their bounds.
template <int P, int DIM, typename T>
__device__ void tail_restrict(const T* rf, int nf, T* bc, T* xc, int nc, const int* rs, const T* rw,
                              int RW) {
    const int nn = nc * nc, Nc = (DIM == 3) ? nn * nc : nn;
    for (int C = threadIdx.x; C < Nc; C += blockDim.x) {
        const int K = C / nn, rem = C - K * nn, J = rem / nc, I = rem - J * nc;
        if constexpr (DIM == 3)
            bc[C] = transfer3d<restrict_bound(P), T>(rf, nf, rs, rw, RW, nc, I, J, K);
        else
            bc[C] = transfer2d<restrict_bound(P), T>(rf, nf, rs, rw, RW, nc, I, J);
        xc[C] = 0;
    }
}

// x_f += P e_c (both in LDS).
template <int P, int DIM, typename T>
__device__ void tail_prolong(const T* ec, int nc, T* xf, int nf, const int* ps, const T* pw, int PW) {
    const int nn = nf * nf, Nf = (DIM == 3) ? nn * nf : nn;
    for (int F = threadIdx.x; F < Nf; F += blockDim.x) {
        const int k = F / nn, rem = F - k * nn, j = rem / nf, i = rem - j * nf;
        if constexpr (DIM == 3)
            xf[F] += transfer3d<prolong_bound(P), T>(ec, nc, ps, pw, PW, nf, i, j, k);
        else
            xf[F] += transfer2d<prolong_bound(P), T>(ec, nc, ps, pw, PW, nf, i, j);
    }
}

// ---- stored 2D stencils: padded LDS layout, vector reads of x --------------

// One stencil row's window of x for a point whose aligned window starts at xw:
// NV vector reads, then the W values from phase S0 (fixed per colour).
template <int P, typename T, int S0>
__device__ __forceinline__ void ft_window(const T* xw, T (&xv)[2 * P + 1]) {
    constexpr int VW = tl_vw(sizeof(T)), NV = tl_nv(P, VW);
    typedef T vec __attribute__((ext_vector_type(VW)));
    T win[NV * VW];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        vec v = *reinterpret_cast<const vec*>(xw + m * VW);
#pragma unroll
        for (int e = 0; e < VW; ++e) win[m * VW + e] = v[e];
    }
#pragma unroll
    for (int a = 0; a < 2 * P + 1; ++a) xv[a] = win[S0 + a];
}

// Gauss-Seidel colour c (mode 0) or residual of colour c (mode 1) on a level
// in the padded layout, one thread per point.  S0 >= 0: the window phase of
// every point of the colour (vector reads); S0 < 0: scalar reads.  The row
// products and their sum follow Stencil2D::slice and the multi-block kernels.
template <int P, typename T, int S0>
__device__ void ft_colour(const Stencil2D<P, T>& A, const T* __restrict__ b, T* xl,
                          T* __restrict__ r, int c, int mode) {
    constexpr int W = 2 * P + 1, S = W * W, VW = tl_vw(sizeof(T)), PADL = tl_padl(P, VW);
    constexpr int VR = (int)sizeof(T) / 4;
    // rows whose loads are in flight together: coefficients and x window of
    // a row take (W + nv*vw) values; keep G rows within 96 VGPRs
    constexpr int G0 = 96 / ((W + tl_nv(P, VW) * VW) * VR);
    constexpr int G = G0 < 1 ? 1 : (G0 > W ? W : G0);
    const int n = A.n, RS = tl_stride(P, VW, n);
    const int ci = c % (P + 1), cj = c / (P + 1);
    const int ni = (n - ci + P) / (P + 1), nj = (n - cj + P) / (P + 1);
    const int cs = ni * nj;
    for (int k = threadIdx.x; k < cs; k += blockDim.x) {
        const int jj = k / ni, ii = k - jj * ni;
        const int i = ci + (P + 1) * ii, j = cj + (P + 1) * jj;
        const long long I = i + (long long)n * j;
        const T bv = as_global(b)[I];
        const auto cf = as_global(A.coef + (size_t)c * S * A.ncp + k);
        const int sc = PADL - P + i;                      // first window column
        const T* xr = xl + (size_t)j * RS + (S0 >= 0 ? sc - S0 : sc);  // padded row j = stencil row 0
        T acc = 0, d = 1;
        // both loops unrolled (w is a constant, no branches); the scheduling
        // barrier keeps the loads of one group of G rows together
#pragma unroll
        for (int w0 = 0; w0 < W; w0 += G) {
            if (w0 > 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int w = w0 + g;
                if (w < W) {
                    T cv[W], xv[W];
#pragma unroll
                    for (int e = 0; e < W; ++e) cv[e] = cf[(size_t)(w * W + e) * A.ncp];
                    if constexpr (S0 >= 0) {
                        ft_window<P, T, S0>(xr + (size_t)w * RS, xv);
                    } else {
#pragma unroll
                        for (int e = 0; e < W; ++e) xv[e] = xr[(size_t)w * RS + e];
                    }
                    T ra = 0;
#pragma unroll
                    for (int e = 0; e < W; ++e) ra = fma(cv[e], xv[e], ra);
                    if (w == P) d = cv[P];
                    acc += ra;
                }
            }
        }
        if (mode == 0) {
            T* xp = xl + (size_t)(j + P) * RS + PADL + i;
            *xp = *xp + (bv - acc) / d;
        } else {
            as_global(r)[I] = bv - acc;
        }
    }
}

// Phase dispatch: the window phase is a function of the colour alone when the
// colour stride p+1 is a multiple of the vector width.
template <int P, typename T, int S0 = 0>
__device__ __forceinline__ void ft_colour_phase(const Stencil2D<P, T>& A, const T* b, T* xl, T* r,
                                                int c, int mode, int s0) {
    constexpr int VW = tl_vw(sizeof(T));
    if constexpr (S0 < VW - 1) {
        if (s0 != S0) {
            ft_colour_phase<P, T, S0 + 1>(A, b, xl, r, c, mode, s0);
            return;
        }
    }
    ft_colour<P, T, S0>(A, b, xl, r, c, mode);
}

template <int P, typename T>
__device__ void ft_pass(const Stencil2D<P, T>& A, const T* __restrict__ b, T* xl,
                        T* __restrict__ r, int c0, int c1, int mode) {
    constexpr int VW = tl_vw(sizeof(T)), PADL = tl_padl(P, VW);
    for (int c = c0; c < c1; ++c) {
        if constexpr ((P + 1) % VW == 0)
            ft_colour_phase<P, T>(A, b, xl, r, c, mode, (PADL - P + c % (P + 1)) % VW);
        else
            ft_colour<P, T, -1>(A, b, xl, r, c, mode);
        if (mode == 0) __syncthreads();
    }
    if (mode == 1) __syncthreads();
}

// b_c = R r_f from memory; the windows are unrolled to their bound.
template <int P, typename T>
__device__ void ft_restrict(const T* __restrict__ rf_, int nf, T* __restrict__ bc_, T* xc, int nc,
                            const int* __restrict__ rs_, const T* __restrict__ rw_, int RW) {
    constexpr int RM = restrict_bound(P), VW = tl_vw(sizeof(T)), PADL = tl_padl(P, VW);
    const int RSc = tl_stride(P, VW, nc);
    const auto rf = as_global(rf_);
    const auto bc = as_global(bc_);
    const auto rs = as_global(rs_);
    const auto rw = as_global(rw_);
    const int last = nc * RW - 1;
    for (int C = threadIdx.x; C < nc * nc; C += blockDim.x) {
        const int I = C % nc, J = C / nc;
        const int i0 = rs[I], j0 = rs[J];
        T wi[RM], wj[RM];
#pragma unroll
        for (int a = 0; a < RM; ++a) {
            wi[a] = (a < RW) ? rw[min(I * RW + a, last)] : (T)0;
            wj[a] = (a < RW) ? rw[min(J * RW + a, last)] : (T)0;
        }
        T s2 = 0;
#pragma unroll
        for (int bq = 0; bq < RM; ++bq) {
            const auto row = rf + (size_t)min(j0 + bq, nf - 1) * nf;
            T s1 = 0;
#pragma unroll
            for (int a = 0; a < RM; ++a) s1 = fma(wi[a], row[min(i0 + a, nf - 1)], s1);
            s2 = fma(wj[bq], s1, s2);
        }
        bc[C] = s2;
        xc[(size_t)(J + P) * RSc + PADL + I] = 0;
    }
}

// x_f += P e_c, both in the padded LDS layout.
template <int P, typename T>
__device__ void ft_prolong(const T* ec, int nc, T* xf, int nf, const int* __restrict__ ps_,
                           const T* __restrict__ pw_, int PW) {
    const auto ps = as_global(ps_);
    const auto pw = as_global(pw_);
    constexpr int PM = prolong_bound(P), VW = tl_vw(sizeof(T)), PADL = tl_padl(P, VW);
    const int RSc = tl_stride(P, VW, nc), RSf = tl_stride(P, VW, nf);
    const int last = nf * PW - 1;
    for (int F = threadIdx.x; F < nf * nf; F += blockDim.x) {
        const int i = F % nf, j = F / nf;
        const int i0 = ps[i], j0 = ps[j];
        T wi[PM], wj[PM];
#pragma unroll
        for (int a = 0; a < PM; ++a) {
            wi[a] = (a < PW) ? pw[min(i * PW + a, last)] : (T)0;
            wj[a] = (a < PW) ? pw[min(j * PW + a, last)] : (T)0;
        }
        T s2 = 0;
#pragma unroll
        for (int bq = 0; bq < PM; ++bq) {
            const T* row = ec + (size_t)(min(j0 + bq, nc - 1) + P) * RSc + PADL;
            T s1 = 0;
#pragma unroll
            for (int a = 0; a < PM; ++a) s1 = fma(wi[a], row[min(i0 + a, nc - 1)], s1);
            s2 = fma(wj[bq], s1, s2);
        }
        xf[(size_t)(j + P) * RSf + PADL + i] += s2;
    }
}

// Prefetching variant (FP32): records rec[(c*ncp + k)*RL + o],
// o = w*W + a, RL = rec_len(p); one point per thread and colour.
typedef float f4v __attribute__((ext_vector_type(4)));

template <int P, int S0>
__device__ __forceinline__ void pf_point(const f4v (&cq)[rec_len(P) / 4], const float* xr, int RS,
                                         float& acc, float& d) {
    constexpr int W = 2 * P + 1;
    acc = 0.f;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        float xv[W];
        if constexpr (S0 >= 0) {
            ft_window<P, float, S0>(xr + (size_t)w * RS, xv);
        } else {
#pragma unroll
            for (int e = 0; e < W; ++e) xv[e] = xr[(size_t)w * RS + e];
        }
        float ra = 0.f;
#pragma unroll
        for (int e = 0; e < W; ++e) ra = fma(cq[(w * W + e) / 4][(w * W + e) % 4], xv[e], ra);
        acc += ra;
    }
    d = cq[(P * W + P) / 4][(P * W + P) % 4];
}

// Register sets of the prefetching sequence: colours c and c + R - 1 are
// loaded into slots c % R and (c + R - 1) % R.  R divides the colour count,
// so a colour uses the same slot in every sweep and the slot of each step is
// known at compile time; R - 1 colours are in flight while one is updated,
// as far as the register file allows (p = 4: none).
template <int P>
constexpr int pf_ring() {
    return P == 1 ? 4 : (P == 2 ? 3 : (P == 3 ? 2 : (P == 4 ? 1 : 2)));
}
template <int P>
struct PfRegs {
    f4v q[rec_len(P) / 4];
    float bv;
    int i, j;
    bool has;
};

// Records, right-hand side value and position of this thread's point of
// colour c.  The loads are unconditional (threads past the colour's points
// load the colour's last record and do not use it), so a wait counts only
// the loads issued before it.
template <int P>
__device__ __forceinline__ void pf_fetch(const Stencil2D<P, float>& A, const float* __restrict__ rec,
                                         const float* __restrict__ b, int c, PfRegs<P>& g) {
    constexpr int RL = rec_len(P), S = (2 * P + 1) * (2 * P + 1);
    const int n = A.n, ci = c % (P + 1), cj = c / (P + 1);
    const int ni = (n - ci + P) / (P + 1), nj = (n - cj + P) / (P + 1);
    const int k = min((int)threadIdx.x, max(ni * nj - 1, 0));
    g.has = (int)threadIdx.x < ni * nj;
    const int jj = k / ni, ii = k - jj * ni;
    g.i = ci + (P + 1) * ii;
    g.j = cj + (P + 1) * jj;
    const float* rp = rec + ((size_t)c * A.ncp + k) * RL;
    const auto src = as_global(reinterpret_cast<const f4v*>(rp));
    // S = (2p+1)^2 = 1 (mod 4): S/4 full vectors and one value (loading the
    // last vector whole would leave loaded values unused, whose registers the
    // compiler reuses at once, making the next use wait for this load)
#pragma unroll
    for (int m = 0; m < S / 4; ++m) g.q[m] = src[m];
    g.q[S / 4][0] = as_global(rp)[S - 1];
    g.bv = as_global(b)[min(g.i + (size_t)n * g.j, (size_t)n * n - 1)];
}

// Colour c (compile time) of a sweep with its prefetched data: Gauss-Seidel
// update (gs) or residual.
template <int P, int C>
__device__ __forceinline__ void pf_colour(const Stencil2D<P, float>& A, float* xl, float* __restrict__ r,
                                          bool gs, const PfRegs<P>& g) {
    constexpr int PADL = tl_padl(P, 4);
    const int n = A.n, RS = tl_stride(P, 4, n);
    if (!g.has) return;
    const int sc = PADL - P + g.i;  // first window column
    float acc, d;
    if constexpr ((P + 1) % 4 == 0) {
        constexpr int S0 = (PADL - P + C % (P + 1)) % 4;  // window phase of the colour
        pf_point<P, S0>(g.q, xl + (size_t)g.j * RS + sc - S0, RS, acc, d);
    } else {
        pf_point<P, -1>(g.q, xl + (size_t)g.j * RS + sc, RS, acc, d);  // scalar window reads
    }
    if (gs) {
        float* xp = xl + (size_t)(g.j + P) * RS + PADL + g.i;
        *xp = *xp + (g.bv - acc) / d;
    } else {
        as_global(r)[g.i + (size_t)n * g.j] = g.bv - acc;
    }
}

// Colours per unrolled group: a multiple of the ring size and of p+1, so that
// the slot and the window phase of a colour are known at compile time.
template <int P>
constexpr int pf_group() {
    constexpr int R = pf_ring<P>();
    int u = P + 1;
    while (u % R != 0) u += P + 1;
    return u;
}

template <int P, bool kSolo, int U = 0>
__device__ __forceinline__ void pf_group_colours(const Stencil2D<P, float>& A, const float* __restrict__ rec,
                                                 const float* __restrict__ b, float* xl,
                                                 float* __restrict__ r, bool gs, int c0,
                                                 PfRegs<P> (&ring)[pf_ring<P>()]) {
    constexpr int NC = (P + 1) * (P + 1), R = pf_ring<P>();
    const int c = c0 + U;
    pf_fetch<P>(A, rec, b, (c + R - 1) % NC, ring[(U + R - 1) % R]);
    pf_colour<P, U>(A, xl, r, gs, ring[U % R]);
    if (gs || c == NC - 1) pf_sync<kSolo>();
    if constexpr (U + 1 < pf_group<P>()) pf_group_colours<P, kSolo, U + 1>(A, rec, b, xl, r, gs, c0, ring);
}

// One sweep: groups of pf_group colours, the groups in a (not unrolled) loop.
template <int P, bool kSolo>
__device__ __forceinline__ void pf_sweep(const Stencil2D<P, float>& A, const float* __restrict__ rec,
                                         const float* __restrict__ b, float* xl, float* __restrict__ r,
                                         bool gs, PfRegs<P> (&ring)[pf_ring<P>()]) {
    constexpr int NC = (P + 1) * (P + 1), R = pf_ring<P>(), U = pf_group<P>();
    static_assert(NC % R == 0 && NC % U == 0 && U % (P + 1) == 0, "colour grouping");
#pragma unroll 1
    for (int c0 = 0; c0 < NC; c0 += U) pf_group_colours<P, kSolo>(A, rec, b, xl, r, gs, c0, ring);
}

// nsw Gauss-Seidel sweeps (an ordering point after every colour), then, if
// resid, r = b - A x over all colours (one at the end), run by the waves that
// hold points.  The records of the next R - 1 colours are in flight while a
// colour is updated, across the LDS-only ordering points (after the last
// colour they fetch colours of a sweep that does not come; the loads are valid
// and unused).
template <int P, bool kSolo>
__device__ void pf_run(const Stencil2D<P, float>& A, const float* __restrict__ rec,
                       const float* __restrict__ b, float* xl, float* __restrict__ r, int nsw, bool resid) {
    constexpr int R = pf_ring<P>();
    const int nsweeps = nsw + (resid ? 1 : 0);
    PfRegs<P> ring[R];
#pragma unroll
    for (int c = 0; c + 1 < R; ++c) pf_fetch<P>(A, rec, b, c, ring[c]);
    for (int sw = 0; sw < nsweeps; ++sw) pf_sweep<P, kSolo>(A, rec, b, xl, r, sw < nsw, ring);
}

// The sequence on a level whose largest colour spans `act` waves: only those
// waves load records and update (one point per thread; inside an active wave
// the lanes past a colour's points load a valid record they do not use, so
// each wait counts exactly the loads issued before it).  The other waves meet
// the same workgroup barriers and nothing else; with act == 1 wave 0 runs
// alone and the workgroup meets once at the end.
template <int P>
__device__ void pf_sequence(const Stencil2D<P, float>& A, const float* __restrict__ rec,
                            const float* __restrict__ b, float* xl, float* __restrict__ r, int nsw,
                            bool resid, int act) {
    constexpr int NC = (P + 1) * (P + 1);
    if (nsw + (resid ? 1 : 0) == 0) return;
    const int wave = threadIdx.x >> 6;
    if (act <= 1) {
        if (wave == 0) pf_run<P, true>(A, rec, b, xl, r, nsw, resid);
        __syncthreads();
        return;
    }
    if (wave < act) {
        pf_run<P, false>(A, rec, b, xl, r, nsw, resid);
    } else {
        const int nbar = nsw * NC + (resid ? 1 : 0);
        for (int k = 0; k < nbar; ++k) __syncthreads();
    }
}

template <int P, typename T>
__device__ void ft_vcycle(const TailArgs<Stencil2D<P, T>>& a) {
    using Op = Stencil2D<P, T>;
    constexpr int VW = tl_vw(sizeof(T)), PADL = tl_padl(P, VW);
    __shared__ __align__(16) T xs[tail_capacity<T>()];
    const int top = a.top;
    const int used = a.xoff[top] + (int)tl_size(P, VW, a.op[top].n);
    for (int e = threadIdx.x; e < used; e += blockDim.x) xs[e] = 0;
    __syncthreads();
    {
        const int n = a.op[top].n, RS = tl_stride(P, VW, n);
        const auto xg = as_global((const T*)a.x[top]);
        T* xt = xs + a.xoff[top];
        for (int I = threadIdx.x; I < n * n; I += blockDim.x)
            xt[(size_t)(I / n + P) * RS + PADL + I % n] = xg[I];
    }
    __syncthreads();
    auto down = [&](int l) {
        const Op& A = a.op[l];
        T* xl = xs + a.xoff[l];
        if constexpr (tail_prefetch<Op>()) {
            pf_sequence<P>(A, a.rec[l], a.b[l], xl, a.r[l], a.nu1, true, a.act[l]);
        } else {
            for (int s = 0; s < a.nu1; ++s) ft_pass(A, a.b[l], xl, a.r[l], 0, Op::NC, 0);
            ft_pass(A, a.b[l], xl, a.r[l], 0, Op::NC, 1);
        }
        ft_restrict<P, T>(a.r[l], A.n, a.b[l - 1], xs + a.xoff[l - 1], a.op[l - 1].n, a.rs[l], a.rw[l],
                          a.RW[l]);
        __syncthreads();
    };
    auto coarse = [&]() {
        const int nc = a.op[0].n, RS = tl_stride(P, VW, nc);
        T* x0 = xs + a.xoff[0];
        const auto b0 = as_global((const T*)a.b[0]);
        const auto Ainv = as_global(a.Ainv);
        for (int r = threadIdx.x; r < a.n0; r += blockDim.x) {
            double s = 0.0;
#pragma unroll 8
            for (int c = 0; c < a.n0; ++c) s = fma(Ainv[(size_t)r * a.n0 + c], (double)b0[c], s);
            x0[(size_t)(r / nc + P) * RS + PADL + r % nc] = (T)s;
        }
        __syncthreads();
    };
    auto up = [&](int l) {
        const Op& A = a.op[l];
        T* xl = xs + a.xoff[l];
        ft_prolong<P, T>(xs + a.xoff[l - 1], a.op[l - 1].n, xl, A.n, a.ps[l], a.pw[l], a.PW[l]);
        __syncthreads();
        if constexpr (tail_prefetch<Op>())
            pf_sequence<P>(A, a.rec[l], a.b[l], xl, a.r[l], a.nu2, false, a.act[l]);
        else
            for (int s = 0; s < a.nu2; ++s) ft_pass(A, a.b[l], xl, a.r[l], 0, Op::NC, 0);
    };
    mu_schedule(top, a.mu, down, coarse, up);
    {
        const int n = a.op[top].n, RS = tl_stride(P, VW, n);
        const auto xg = as_global(a.x[top]);
        const T* xt = xs + a.xoff[top];
        for (int I = threadIdx.x; I < n * n; I += blockDim.x)
            xg[I] = xt[(size_t)(I / n + P) * RS + PADL + I % n];
    }
}

// ---- sum-factorised operators: natural layout ------------------------------

// ---- sum-factorised levels in the single-workgroup kernel ------------------
//
// Row-class Gauss-Seidel as in k_gs_rowclass_kron with x in LDS: one wave per
// x-row of the class (n <= 64, one lane per point), the rows of a class spread
// over the workgroup's waves.  A row's p+1 colour steps touch only its own
// row, so they are ordered by the wave's own LDS operations; each class ends
// with one workgroup barrier.  The neighbours' u, v come from the other lanes
// by cross-lane reads.  The arithmetic is that of the multi-block kernels
// (same contraction, same summation order), so both give the same iterates.
constexpr int kTailKronMaxN = 64;

// sum_a Kx_{i,a} u_{i+a} + Mx_{i,a} v_{i+a} for the lane's point i (its band
// rows kxr, mxr, each entry read at its use); lanes outside the row hold
// u = v = 0 and out-of-row offsets have zero band entries.  cr (optional)
// receives the in-row coupling m00 Kx_{i,a} + g00 Mx_{i,a}.
template <int W, typename T>
__device__ __forceinline__ T tail_kron_xproduct(const T* kxr, const T* mxr, T u, T v, int lane, T m00, T g00,
                                                T* cr) {
    constexpr int P = (W - 1) / 2;
    T acc = 0;
#pragma unroll
    for (int a = 0; a < W; ++a) {
        const int src = clampi(lane + a - P, 0, 63);
        const T kx = kxr[a], mx = mxr[a];
        acc = fma(kx, __shfl(u, src, 64), acc);
        acc = fma(mx, __shfl(v, src, 64), acc);
        if (cr) cr[a] = fma(m00, kx, g00 * mx);
    }
    return acc;
}

// gs: one multicolour Gauss-Seidel sweep of the level in row classes; else
// r = b - A x on every point (x unchanged).  Ends with a workgroup barrier.
template <class Op>
__device__ void tail_rows_kron(const Op& A, const typename Op::T* __restrict__ b, typename Op::T* x,
                               typename Op::T* __restrict__ r, bool gs) {
    using T = typename Op::T;
    constexpr int P = Op::kP, W = Op::W, DIM = is_kron3<Op>() ? 3 : 2;
    const int n = A.n, NWAVE = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i = min(lane, n - 1);
    // the lane's x band rows: read from LDS at their use (2D, where registers
    // are short at high degree) or loaded after each contraction (3D)
    T kxa[W], mxa[W];
    const T* kxr = A.K + i * W;
    const T* mxr = A.M + i * W;
    auto xbands = [&]() {
        if constexpr (DIM == 3) {
#pragma unroll
            for (int a = 0; a < W; ++a) {
                kxa[a] = A.K[i * W + a];
                mxa[a] = A.M[i * W + a];
            }
        }
    };
    const T* kxp = (DIM == 3) ? kxa : kxr;
    const T* mxp = (DIM == 3) ? mxa : mxr;
    if (!gs) {
        const int rows = (DIM == 3) ? n * n : n;
        for (int row = wave; row < rows; row += NWAVE) {
            const int k = row / n, j = row - k * n;  // k = 0 in 2D
            T u, v;
            kron_row_contract<Op, true, false>(A, x, j, k, i, u, v);
            if (lane >= n) u = v = 0;
            xbands();
            const T acc = tail_kron_xproduct<W, T>(kxp, mxp, u, v, lane, (T)0, (T)0, (T*)nullptr);
            if (lane < n) r[(size_t)row * n + lane] = b[(size_t)row * n + lane] - acc;
        }
        __syncthreads();
        return;
    }
    const int s_own = lane % (P + 1);
    for (int ck = 0; ck <= (DIM == 3 ? P : 0); ++ck)
        for (int cj = 0; cj <= P; ++cj) {
            const int nj = (n - cj + P) / (P + 1), nk = (DIM == 3) ? (n - ck + P) / (P + 1) : 1;
            for (int rr = wave; rr < nj * nk; rr += NWAVE) {
                const int kq = rr / nj, jq = rr - kq * nj;
                const int j = cj + (P + 1) * jq, k = ck + (P + 1) * kq;
                const size_t row = kron_row_offset<Op>(n, j, k);
                T* xr = x + row;
                const T bo = b[row + i];
                T u, v;
                kron_row_contract<Op, false, false>(A, x, j, k, i, u, v);
                if (lane >= n) u = v = 0;
                T m00, g00;
                kron_row_self(A, j, k, m00, g00);
                T cr[W];
                xbands();
                const T rest = tail_kron_xproduct<W, T>(kxp, mxp, u, v, lane, m00, g00, cr);
#pragma unroll
                for (int s = 0; s <= P; ++s) {
                    if (lane < n && s_own == s) {
                        T acc = rest;
#pragma unroll
                        for (int a = 0; a < W; ++a) acc = fma(cr[a], xr[clampi(lane + a - P, 0, n - 1)], acc);
                        xr[lane] = xr[lane] + (bo - acc) / cr[P];
                    }
                    pf_sync<true>();
                }
            }
            __syncthreads();
        }
}

// mu-cycle (Algorithm 2) on levels 0..top with right-hand side b[top] and
// iterate x[top] (in place), by one workgroup.  LDS holds, level by
// level, the 1D bands K and M (levels >= 1, at boff) and the iterate (at
// xoff), then kTailPadVals zeros; the host checks that this fits and that
// every level has at most kTailKronMaxN unknowns per direction (one wave per
// row of a row class).
template <class Op>
__device__ void gt_vcycle(const TailArgs<Op>& a) {
    using T = typename Op::T;
    constexpr int DIM = std::is_same<typename Op::Pt, Pt3>::value ? 3 : 2;
    constexpr int P = Op::kP, W = Op::W;
    __shared__ T xs[tail_capacity<T>()];
    const int top = a.top;
    for (int l = 1; l <= top; ++l) {
        const int nw = a.op[l].n * W;
        T* kb = xs + a.boff[l];
        for (int e = threadIdx.x; e < nw; e += blockDim.x) {
            kb[e] = a.op[l].K[e];
            kb[nw + e] = a.op[l].M[e];
        }
    }
    {
        const T* xg = a.x[top];
        T* xt = xs + a.xoff[top];
        const int Nt = (int)a.N[top];
        for (int i = threadIdx.x; i < Nt + kTailPadVals; i += blockDim.x) xt[i] = (i < Nt) ? xg[i] : (T)0;
    }
    __syncthreads();
    // operator of level l reading its bands from LDS
    auto lop = [&](int l) {
        Op A = a.op[l];
        A.K = xs + a.boff[l];
        A.M = A.K + A.n * W;
        return A;
    };
    auto down = [&](int l) {
        const Op A = lop(l);
        T* xl = xs + a.xoff[l];
        for (int s = 0; s < a.nu1; ++s) tail_rows_kron(A, a.b[l], xl, a.r[l], true);
        tail_rows_kron(A, a.b[l], xl, a.r[l], false);
        tail_restrict<P, DIM, T>(a.r[l], A.n, a.b[l - 1], xs + a.xoff[l - 1], a.op[l - 1].n, a.rs[l],
                                 a.rw[l], a.RW[l]);
        __syncthreads();
    };
    auto coarse = [&]() {
        T* x0 = xs + a.xoff[0];
        const T* b0 = a.b[0];
        for (int r = threadIdx.x; r < a.n0; r += blockDim.x) {
            double s = 0.0;
#pragma unroll 8
            for (int c = 0; c < a.n0; ++c) s = fma(a.Ainv[(size_t)r * a.n0 + c], (double)b0[c], s);
            x0[r] = (T)s;
        }
        __syncthreads();
    };
    auto up = [&](int l) {
        const Op A = lop(l);
        T* xl = xs + a.xoff[l];
        tail_prolong<P, DIM, T>(xs + a.xoff[l - 1], a.op[l - 1].n, xl, A.n, a.ps[l], a.pw[l], a.PW[l]);
        __syncthreads();
        for (int s = 0; s < a.nu2; ++s) tail_rows_kron(A, a.b[l], xl, a.r[l], true);
    };
    mu_schedule(top, a.mu, down, coarse, up);
    {
        T* xg = a.x[top];
        const T* xt = xs + a.xoff[top];
        for (long long i = threadIdx.x; i < a.N[top]; i += blockDim.x) xg[i] = xt[i];
    }
}

template <class Op>
__device__ __forceinline__ void vcycle_tail_body(const TailArgs<Op>& a) {
    if constexpr (Op::kColourOrder)
        ft_vcycle<Op::kP, typename Op::T>(a);
    else
        gt_vcycle(a);
}

template <class Op>
__global__ void __launch_bounds__(tail_threads<Op>()) k_vcycle_tail(TailArgs<Op> a) {
    vcycle_tail_body(a);
}

// Batched: workgroup e runs problem e's small-level V-cycle.
template <class Op>
__global__ void __launch_bounds__(tail_threads<Op>()) k_b_tail(const TailArgs<Op>* __restrict__ A) {
    vcycle_tail_body(A[blockIdx.x]);
}

// Per-point coefficient records of a level for the prefetching tail:
// rec[(c*ncp + k)*RL + o] = coef[(c*S + o)*ncp + k] for o < S, zero padding.
template <int P>
__global__ void k_to_records(const float* __restrict__ coef, int ncp, int ncol, float* __restrict__ rec) {
    constexpr int S = (2 * P + 1) * (2 * P + 1), RL = rec_len(P);
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= (long long)ncol * ncp * RL) return;
    const int o = (int)(t % RL);
    const long long ck = t / RL;
    const int k = (int)(ck % ncp), c = (int)(ck / ncp);
    rec[t] = (o < S) ? coef[((size_t)c * S + o) * ncp + k] : 0.f;
}

// ---------------------------------------------------------------------------
// setup kernels (FP64): mapped assembly of the finest stencil, load vector,
// Galerkin products on stencils, colour-blocked layout

// Geometry and coefficients of a 2D problem assembled from quadrature.
// kind 0: unit square (identity map); 1: quarter annulus as the polynomial
// degree-2 B-spline surface on one element with control net
// rho_a * {(1,0), (1,1), (0,1)}_b, rho = (r_in, (r_in + r_out)/2, r_out);
// 2: the same net with weights (1, 1/sqrt 2, 1) in eta (rational quadratic,
// exact circular arcs).  pde 0: -Laplace; 1, 2: -div(A grad u) + B.grad u + c u
// with the two coefficient sets of Section 4.3 (unit square: B of its first
// problem, c = 1; quarter annulus: B = (-5y, 5x), c = xy; the same A); 3: the
// advection-diffusion problem of Section 4.3, A = 0.1 I, B = (1, 1), c = 0.
struct GeomParams {
    int kind;
    int pde;
    double r_in, r_out;
};

// At every quadrature point: w |det J| J^-1 A J^-T (D11, D12, D22; A = I for
// the Laplace operator), w |det J| (for loads), the physical point, and for
// pde > 0 the reference convection w |det J| J^-1 B (Bx, By) and w |det J| c.
struct GeomQP {
    double* D11;
    double* D12;
    double* D22;
    double* wdet;
    double* X;
    double* Y;
    double* Bx;  // null for pde 0
    double* By;
    double* Cw;
};

// Coefficients of the Section 4.3 problems at a physical point (pde 1, 2 or 3).
__device__ inline void pde_coefficients(int pde, double x, double y, double& a11, double& a12, double& a22,
                                        double& b1, double& b2, double& c) {
    if (pde == 3) {  // advection-diffusion: -0.1 Laplace + (1, 1) . grad
        a11 = a22 = 0.1;
        a12 = 0.0;
        b1 = b2 = 1.0;
        c = 0.0;
        return;
    }
    a11 = (2.0 + cos(x)) * (1.0 + y);
    a12 = cos(x + y) * sin(x + y);
    a22 = (2.0 + sin(y)) * (1.0 + x);
    if (pde == 1) {
        const double cc = cos(x + y) * cos(x + y);
        b1 = 11.0 + sin(x) + y * sin(x) - 2.0 * cc;
        b2 = -9.0 - cos(y) - x * cos(y) - 2.0 * cc;
        c = 1.0;
    } else {
        b1 = -5.0 * y;
        b2 = 5.0 * x;
        c = x * y;
    }
}

__device__ inline void bernstein2(double u, double* B, double* dB) {
    B[0] = (1 - u) * (1 - u);
    B[1] = 2 * u * (1 - u);
    B[2] = u * u;
    dB[0] = -2 * (1 - u);
    dB[1] = 2 - 4 * u;
    dB[2] = 2 * u;
}

__global__ void k_geometry_qp(GeomParams gp, int NQ, const double* __restrict__ pts,
                              const double* __restrict__ wts, GeomQP G) {
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)NQ * NQ) return;
    int qy = (int)(t / NQ), qx = (int)(t - (long long)qy * NQ);
    double xi = pts[qx], eta = pts[qy];
    double J00, J01, J10, J11, X, Y;
    if (gp.kind == 1) {
        const double rho[3] = {gp.r_in, 0.5 * (gp.r_in + gp.r_out), gp.r_out};
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
    } else if (gp.kind == 2) {
        // rho(xi) C(eta), C = sum_b w_b B_b (eta) P_b / sum_b w_b B_b(eta)
        const double rho[3] = {gp.r_in, 0.5 * (gp.r_in + gp.r_out), gp.r_out};
        const double cx[3] = {1.0, 1.0, 0.0}, cy[3] = {0.0, 1.0, 1.0};
        const double wb[3] = {1.0, 0.70710678118654752440, 1.0};
        double Bu[3], dBu[3], Bv[3], dBv[3];
        bernstein2(xi, Bu, dBu);
        bernstein2(eta, Bv, dBv);
        double r = 0.0, dr = 0.0, nx = 0.0, ny = 0.0, dnx = 0.0, dny = 0.0, den = 0.0, dden = 0.0;
        for (int a = 0; a < 3; ++a) {
            r += Bu[a] * rho[a];
            dr += dBu[a] * rho[a];
        }
        for (int b = 0; b < 3; ++b) {
            nx += wb[b] * Bv[b] * cx[b];
            ny += wb[b] * Bv[b] * cy[b];
            dnx += wb[b] * dBv[b] * cx[b];
            dny += wb[b] * dBv[b] * cy[b];
            den += wb[b] * Bv[b];
            dden += wb[b] * dBv[b];
        }
        const double Cx = nx / den, Cy = ny / den;
        const double dCx = (dnx - Cx * dden) / den, dCy = (dny - Cy * dden) / den;
        X = r * Cx;
        Y = r * Cy;
        J00 = dr * Cx;
        J01 = r * dCx;
        J10 = dr * Cy;
        J11 = r * dCy;
    } else {
        X = xi;
        Y = eta;
        J00 = 1.0;
        J01 = 0.0;
        J10 = 0.0;
        J11 = 1.0;
    }
    double det = J00 * J11 - J01 * J10;
    double w = wts[qx] * wts[qy] * fabs(det);
    if (gp.pde == 0) {
        double a = J00 * J00 + J10 * J10, b = J00 * J01 + J10 * J11, c = J01 * J01 + J11 * J11;
        double id = 1.0 / (a * c - b * b);
        G.D11[t] = w * c * id;
        G.D12[t] = -w * b * id;
        G.D22[t] = w * a * id;
    } else {
        // J^-1 = [[J11, -J01], [-J10, J00]] / det; K = J^-1 A J^-T, bh = J^-1 B
        double a11, a12, a22, b1, b2, cr;
        pde_coefficients(gp.pde, X, Y, a11, a12, a22, b1, b2, cr);
        const double i00 = J11 / det, i01 = -J01 / det, i10 = -J10 / det, i11 = J00 / det;
        const double m00 = i00 * a11 + i01 * a12, m01 = i00 * a12 + i01 * a22;  // J^-1 A
        const double m10 = i10 * a11 + i11 * a12, m11 = i10 * a12 + i11 * a22;
        G.D11[t] = w * (m00 * i00 + m01 * i01);
        G.D12[t] = w * (m00 * i10 + m01 * i11);
        G.D22[t] = w * (m10 * i10 + m11 * i11);
        G.Bx[t] = w * (i00 * b1 + i01 * b2);
        G.By[t] = w * (i10 * b1 + i11 * b2);
        G.Cw[t] = w * cr;
    }
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
                        if (G.Bx) {  // (B . grad phi_{I+o}) phi_I + c phi_{I+o} phi_I
                            const double v1 = vi * vj, v2 = vi2 * vj2;
                            acc += (G.Bx[qi] * gx2 + G.By[qi] * gy2) * v1 + G.Cw[qi] * v1 * v2;
                        }
                    }
            }
    }
    out[t] = acc;
}

// Built-in right-hand sides of the Section 4.3 problems at the quadrature points,
// premultiplied by w |det J|: pde 1 and 3: f = 1; pde 2: f of the manufactured solution
// u = (x^2 + y^2 - 0.2^2)(x^2 + y^2 - 1) sin x sin y, i.e.
// f = -div(A grad u) + B.grad u + c u written out with u = g s,
// g = (r^2 - 0.04)(r^2 - 1), s = sin x sin y.
__global__ void k_load_qp_builtin(long long nqp, GeomQP G, int pde, double* __restrict__ fq) {
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nqp) return;
    const double x = G.X[t], y = G.Y[t];
    double f = 1.0;
    if (pde == 2) {
        const double r2 = x * x + y * y, h = 2.0 * r2 - 1.04, g = (r2 - 0.04) * (r2 - 1.0);
        const double gx = 2.0 * x * h, gy = 2.0 * y * h;
        const double gxx = 8.0 * x * x + 2.0 * h, gyy = 8.0 * y * y + 2.0 * h, gxy = 8.0 * x * y;
        const double sxv = sin(x), cxv = cos(x), syv = sin(y), cyv = cos(y);
        const double s = sxv * syv, sx = cxv * syv, sy = sxv * cyv, sxy = cxv * cyv;
        const double u = g * s, ux = gx * s + g * sx, uy = gy * s + g * sy;
        const double uxx = gxx * s + 2.0 * gx * sx - g * s, uyy = gyy * s + 2.0 * gy * sy - g * s;
        const double uxy = gxy * s + gx * sy + gy * sx + g * sxy;
        double a11, a12, a22, b1, b2, c;
        pde_coefficients(2, x, y, a11, a12, a22, b1, b2, c);
        const double a11x = -sxv * (1.0 + y), a12d = cos(2.0 * (x + y)), a22y = cyv * (1.0 + x);
        const double div = a11x * ux + a11 * uxx + a12d * uy + 2.0 * a12 * uxy + a12d * ux + a22y * uy +
                           a22 * uyy;
        f = -div + b1 * ux + b2 * uy + c * u;
    }
    fq[t] = f * G.wdet[t];
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
// Exact symmetry of an assembled stencil operator (natural layout, n^2 rows
// of S offsets): every lower-half entry A[I, I+o] (offsets before the centre,
// o < p W + p) takes the value of its mirror A[J, J-o], J = I + o, an
// upper-half entry, so that A equals A^T bit for bit (assembly and Galerkin
// products give it up to rounding).
template <int P>
__global__ void k_symmetrize_stencil(double* __restrict__ st, int n) {
    constexpr int W = 2 * P + 1, S = W * W, H0 = P * W + P;
    long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)n * n * H0) return;
    const long long I = t / H0;
    const int o = (int)(t - I * H0);
    const int j = (int)(I / n), i = (int)(I - (long long)j * n);
    const int i2 = i + o % W - P, j2 = j + o / W - P;
    if (i2 < 0 || i2 >= n || j2 < 0 || j2 >= n) return;
    st[I * S + o] = st[((long long)j2 * n + i2) * S + (S - 1 - o)];
}

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
