// Batched kernels: one launch covers the same step of many independent
// problems.  Each launch gets a table of per-problem entries and the prefix
// offsets of their block counts; a block finds its problem by binary search.
#pragma once

#include "kernels.hpp"

namespace igamg {

__device__ __forceinline__ int bmap_find(const int* __restrict__ offs, int ne, int bid) {
    int lo = 0, hi = ne;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (offs[mid] <= bid) lo = mid; else hi = mid;
    }
    return lo;
}

template <class Op>
struct BGs {
    Op op;
    const typename Op::T* b;
    typename Op::T* x;
};

// offs: (NC rows of ne+1 prefix block counts), row c used for colour c
template <class Op>
__global__ void __launch_bounds__(64 * Op::NW) k_b_gs(const BGs<Op>* __restrict__ E,
                                                      const int* __restrict__ offs, int ne, int c) {
    const int* o = offs + (size_t)c * (ne + 1);
    int e = bmap_find(o, ne, blockIdx.x);
    const BGs<Op> en = E[e];
    gs_colour_body(en.op, en.b, en.x, c, blockIdx.x - o[e]);
}

// Row-class sweep step of many problems: offs holds, per class r, the prefix
// counts of the problems' rows in that class; a workgroup runs one row
// (workgroups of one problem's rows are consecutive, in XCD order).
template <class Op, bool kStream>
__global__ void __launch_bounds__(kRowThreads) k_b_rowclass(const BGs<Op>* __restrict__ E,
                                                            const int* __restrict__ offs, int ne, int r) {
    const int* o = offs + (size_t)r * (ne + 1);
    const int blk = xcd_swizzle(blockIdx.x, gridDim.x);
    const int e = bmap_find(o, ne, blk);
    const BGs<Op> en = E[e];
    rowclass_body<Op, kStream>(en.op, en.b, en.x, r, blk - o[e]);
}

template <class Op, typename Tout>
struct BRes {
    Op op;
    const typename Op::T* b;
    const typename Op::T* x;
    Tout* out;
    long long N;
};

template <class Op, typename Tout>
__global__ void __launch_bounds__(64 * Op::NW) k_b_res(const BRes<Op, Tout>* __restrict__ E,
                                                       const int* __restrict__ offs, int ne) {
    int e = bmap_find(offs, ne, blockIdx.x);
    const BRes<Op, Tout> en = E[e];
    residual_body<Op, Tout>(en.op, en.b, en.x, en.out, 0, 0.0, en.N, nullptr, blockIdx.x - offs[e], 0);
}

template <typename T>
struct BTr {
    const T* src;
    T* dst;
    T* zero;
    int nf, nc;
    const int* st;
    const T* w;
    int W;
};

// restriction (dst = R src on the coarse grid, zero <- 0)
template <int P, typename T>
__global__ void __launch_bounds__(kBlock) k_b_restrict(const BTr<T>* __restrict__ E,
                                                       const int* __restrict__ offs, int ne) {
    int e = bmap_find(offs, ne, blockIdx.x);
    const BTr<T> en = E[e];
    long long C = (long long)(blockIdx.x - offs[e]) * kBlock + threadIdx.x;
    int nc = en.nc, nf = en.nf;
    if (C >= (long long)nc * nc) return;
    en.zero[C] = 0;
    int J = (int)(C / nc), I = (int)(C - (long long)J * nc);
    en.dst[C] = transfer2d<restrict_bound(P), T>(en.src, nf, en.st, en.w, en.W, nc, I, J);
}

// prolongation and correction (dst += P src), src coarse, dst fine
template <int P, typename T>
__global__ void __launch_bounds__(kBlock) k_b_prolong(const BTr<T>* __restrict__ E,
                                                      const int* __restrict__ offs, int ne) {
    int e = bmap_find(offs, ne, blockIdx.x);
    const BTr<T> en = E[e];
    long long F = (long long)(blockIdx.x - offs[e]) * kBlock + threadIdx.x;
    int nc = en.nc, nf = en.nf;
    if (F >= (long long)nf * nf) return;
    int j = (int)(F / nf), i = (int)(F - (long long)j * nf);
    en.dst[F] += transfer2d<prolong_bound(P), T>(en.src, nc, en.st, en.w, en.W, nf, i, j);
}

template <typename T>
struct BCoarse {
    const double* Ainv;
    int n0;
    const T* b;
    T* x;
};

// one block per problem
template <typename T>
__global__ void __launch_bounds__(kBlock) k_b_coarse(const BCoarse<T>* __restrict__ E) {
    const BCoarse<T> en = E[blockIdx.x];
    for (int r = threadIdx.x; r < en.n0; r += kBlock) {
        double s = 0.0;
        for (int c = 0; c < en.n0; ++c) s = fma(en.Ainv[(size_t)r * en.n0 + c], (double)en.b[c], s);
        en.x[r] = (T)s;
    }
}

struct BVec {
    const double* a64;
    double* b64;
    float* f32;
    long long N;
};

// mode 0: f32 = 0; mode 1: b64 = a64; mode 2: b64 += f32
__global__ void __launch_bounds__(kBlock) k_b_vec(const BVec* __restrict__ E, const int* __restrict__ offs,
                                                  int ne, int mode) {
    int e = bmap_find(offs, ne, blockIdx.x);
    const BVec en = E[e];
    long long I = (long long)(blockIdx.x - offs[e]) * kBlock + threadIdx.x;
    if (I >= en.N) return;
    if (mode == 0)
        en.f32[I] = 0.f;
    else if (mode == 1)
        en.b64[I] = en.a64[I];
    else
        en.b64[I] += (double)en.f32[I];
}

// dst[e] = *src[e]
__global__ void k_b_gather(const double* const* __restrict__ src, int ne, double* __restrict__ dst) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ne) dst[e] = *src[e];
}

}  // namespace igamg
