// Extrapolated geometric multigrid for B-spline IGA Poisson problems on
// MI355X: context, setup, V-cycle orchestration, restarted RRE/MPE driver and
// the C ABI declared in include/igamg.h.
//
// Method: arXiv 2412.20205 -- Algorithm 2 (mu-cycle, mu = 1) as the fixed-point
// map G of eq. (7), Algorithms 3/4 (RRE/MPE by QR of the differences) and
// Algorithm 5 (restarted extrapolation); Galerkin coarse operators eq. (4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/igamg.h"
#include "common.hpp"
#include "host_spline.hpp"
#include "kernels.hpp"
#include "learned.hpp"
#include "batch.hpp"
#include "solve1d.hpp"

using namespace igamg;

namespace {

// Tall-skinny QR tree of Delta S (iterates it[0..q+1], N unknowns) and the
// small RRE/MPE solve of Algorithms 3/4, enqueued on `stream`: leaf R factors
// go to R0 (ceil(N / kQrRows) blocks of (q+1)^2 doubles), the tree levels
// ping-pong between R0 and R1 (R1 holds ceil(leaves / (kQrRows / (q+1)))
// blocks), the coefficients to `out` (device).
void tsqr_coeffs_async(hipStream_t stream, const IterPtrs& it, int q, long long N, int method,
                       double* R0, double* R1, ExtrapCoeffs* out) {
    const int ncols = q + 1;
    long long count = (N + kQrRows - 1) / kQrRows;
    const size_t shm = (size_t)kQrRows * ncols * sizeof(double);
    hipLaunchKernelGGL(k_tsqr_leaf, dim3((unsigned)count), dim3(kBlock), shm, stream, it, ncols, N, R0);
    IGAMG_HIP(hipGetLastError());
    double* R[2] = {R0, R1};
    int cur = 0;
    const int group = kQrRows / ncols;
    while (count > 1) {
        long long nxt = (count + group - 1) / group;
        size_t shm2 = (size_t)group * ncols * ncols * sizeof(double);
        hipLaunchKernelGGL(k_tsqr_node, dim3((unsigned)nxt), dim3(kBlock), shm2, stream, R[cur],
                           (int)count, group, ncols, R[1 - cur]);
        IGAMG_HIP(hipGetLastError());
        cur = 1 - cur;
        count = nxt;
    }
    hipLaunchKernelGGL(k_extrap_coeffs, dim3(1), dim3(64), 0, stream, R[cur], ncols, method, out);
    IGAMG_HIP(hipGetLastError());
}

thread_local std::string g_last_error;

// Autotuned launch shapes of one problem (key: architecture, geometry,
// operator, degree, grid, precision), process-wide: the split between
// multi-block levels and the single-workgroup kernel, and per level the sweep
// launch shape and the learned inference kernel.
struct TuneChoice {
    int tail_items = 32;
    std::vector<int> row;      // 1: row-class sweeps where available; 0: one launch per colour
    std::vector<int> learned;  // learned inference kernel (igamg_ctx::learned_apply)
    double vcycle_ms = 0.0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;

enum OpKind { OP_STENCIL2D = 0, OP_KRON2D = 1, OP_KRON3D = 2 };

inline unsigned grid_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct Level {
    int n_el = 0, n = 0;
    long long N = 0;
    int ncol = 0, ncp = 0;
    double* coef64 = nullptr;
    float* coef32 = nullptr;
    float* rec32 = nullptr;  // per-point FP32 coefficient records for the prefetching tail
    double *K64 = nullptr, *M64 = nullptr;
    float *K32 = nullptr, *M32 = nullptr;
    Band1D Kh, Mh;
    int *r_start = nullptr, *p_start = nullptr;
    double *r_w64 = nullptr, *p_w64 = nullptr;
    float *r_w32 = nullptr, *p_w32 = nullptr;
    int RW = 0, PW = 0;
    bool sym = false;        // stored stencils made exactly symmetric at setup
    double *x64 = nullptr, *b64 = nullptr, *r64 = nullptr;
    float *x32 = nullptr, *b32 = nullptr, *r32 = nullptr;

    template <typename T> T* x() { if constexpr (std::is_same_v<T, double>) return x64; else return x32; }
    template <typename T> T* b() { if constexpr (std::is_same_v<T, double>) return b64; else return b32; }
    template <typename T> T* r() { if constexpr (std::is_same_v<T, double>) return r64; else return r32; }
    template <typename T> const T* rw() const { if constexpr (std::is_same_v<T, double>) return r_w64; else return r_w32; }
    template <typename T> const T* pw() const { if constexpr (std::is_same_v<T, double>) return p_w64; else return p_w32; }
    template <typename T> const T* coef() const { if constexpr (std::is_same_v<T, double>) return coef64; else return coef32; }
    template <typename T> const T* Kb() const { if constexpr (std::is_same_v<T, double>) return K64; else return K32; }
    template <typename T> const T* Mb() const { if constexpr (std::is_same_v<T, double>) return M64; else return M32; }
};

int colour_size_host(int n, int p, int dim, int c) {
    int s = 1;
    for (int d = 0; d < dim; ++d) {
        int cd = c % (p + 1);
        c /= (p + 1);
        s *= (n - cd + p) / (p + 1);
    }
    return s;
}

}  // namespace

struct igamg_ctx {
    int geom = 0, p = 0, dim = 2, L = 0;
    double r_in = 1.0, r_out = 2.0;  // annulus radii
    // geometry and operator for the quadrature kernels
    GeomParams geom_params() const {
        GeomParams g;
        g.kind = geom == IGAMG_QUARTER_ANNULUS ? 1 : (geom == IGAMG_QUARTER_ANNULUS_EXACT ? 2 : 0);
        g.pde = opt.pde;
        g.r_in = r_in;
        g.r_out = r_out;
        return g;
    }
    bool assembled() const {  // stored stencil assembled from quadrature
        return geom == IGAMG_QUARTER_ANNULUS || geom == IGAMG_QUARTER_ANNULUS_EXACT || opt.pde != 0;
    }
    OpKind kind = OP_STENCIL2D;
    igamg_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<Level> lv;
    std::vector<void*> allocs;
    double* Ainv0 = nullptr;
    int n0 = 0;
    double* b = nullptr;
    double bnorm = 0.0;
    double* partial = nullptr;
    long long npartial = 0;
    double* scal = nullptr;       // device scalars: [0] relative residual, [1] ||b||
    double* host_scal = nullptr;  // pinned
    std::vector<double*> S;       // iterate buffers
    double* Rbuf[2] = {nullptr, nullptr};
    size_t Rcap = 0;
    ExtrapCoeffs* coeffs = nullptr;
    ExtrapCoeffs* host_coeffs = nullptr;
    // element tables of the finest level (2D assembly / loads)
    double *tabV = nullptr, *tabD = nullptr, *tabPts = nullptr, *tabWts = nullptr;
    int nq = 0;
    double setup_ms = 0.0;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_method = -1, graph_q = -1;
    bool graph_resnorm = true;          // the captured cycle ends with ||b - A t||
    // flexible GMRES work space
    std::vector<double*> kry_V, kry_Z;
    double* kry_w = nullptr;
    double* kry_h = nullptr;
    double* kry_partial = nullptr;
    double* bsave = nullptr;
    // checkpoint of the last restarted solve: the accepted iterate (also the
    // iterate a restart cycle started from, while it runs) and its counters;
    // a state loaded by igamg_set_state for the next solve
    double* ckpt = nullptr;
    bool have_state = false;
    igamg_state state{};
    bool resume = false;
    igamg_state resume_state{};
    ExtrapCoeffs last_coeffs{};          // of the last extrapolation read back
    bool have_coeffs = false;
    int tail_top = 0;  // levels 0..tail_top run in the single-workgroup kernel
    bool tail_auto = false;  // tail_items < 0 at setup: take the tuned split of each precision
    // learned smoother
    struct Net {
        bool have = false;
        bool on = true;  // used by the V-cycle (training may turn a level's network off)
        uint16_t *wc = nullptr, *w2f = nullptr, *w2b = nullptr;
        float* mf32 = nullptr;       // per-lane MFMA records of the inference kernel
        uint16_t* mfbf = nullptr;
        float *master = nullptr, *m = nullptr, *v = nullptr;
    };
    std::vector<Net> nets;
    std::vector<double*> diag64;
    std::vector<float*> diag32;
    float* lz = nullptr;       // z = D^{-1} r of the current level (FP32)
    bool learned_on = false;
    // per level: learned inference kernel (learned_apply) and sweep launch
    // shape (row_sweeps); defaults, or the tuned choice
    std::vector<int> learned_kern;
    std::vector<int> row_pref;
    double tuned_ms = 0.0;
    double rho_plain_ref = 0.0;  // measured plain contraction (fallback threshold)

    ~igamg_ctx() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void* a : allocs) (void)hipFree(a);
        if (host_scal) (void)hipHostFree(host_scal);
        if (host_coeffs) (void)hipHostFree(host_coeffs);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    template <typename T>
    T* alloc(size_t count) {
        void* p = nullptr;
        if (count == 0) count = 1;
        if (hipMalloc(&p, count * sizeof(T)) != hipSuccess)
            throw Error(IGAMG_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
        allocs.push_back(p);
        return (T*)p;
    }
    // FP32 iterate vector with kXPad zeros before and after (the FP32 stencil
    // kernels read stencil rows unclamped); never released before the context.
    float* alloc_padded32(long long n) {
        float* base = alloc<float>((size_t)n + 2 * kXPad);
        fill(base, n + 2 * kXPad);
        return base + kXPad;
    }
    void release(void* p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        (void)hipFree(p);
    }
    template <typename T>
    T* upload(const std::vector<T>& v) {
        T* d = alloc<T>(v.size());
        IGAMG_HIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream));
        return d;
    }
    void check_launch() { IGAMG_HIP(hipGetLastError()); }
    template <typename T>
    void fill(T* p, long long n) {
        if (n <= 0) return;
        hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kBlock), 0, stream, p, (T)0, n);
        check_launch();
    }
    template <typename A, typename B>
    void copy(const A* a, B* b, long long n) {
        if (n <= 0) return;
        hipLaunchKernelGGL((k_copy<A, B>), dim3(grid_for(n)), dim3(kBlock), 0, stream, a, b, n);
        check_launch();
    }

    // ---- degree dispatch
    template <class F>
    void with_p(F&& f) {
        switch (p) {
            case 1: f(std::integral_constant<int, 1>{}); break;
            case 2: f(std::integral_constant<int, 2>{}); break;
            case 3: f(std::integral_constant<int, 3>{}); break;
            case 4: f(std::integral_constant<int, 4>{}); break;
            case 5: f(std::integral_constant<int, 5>{}); break;
            default: throw Error(IGAMG_EINVAL, "degree must be 1..5");
        }
    }
    template <class F>
    void with_p3(F&& f) {
        switch (p) {
            case 1: f(std::integral_constant<int, 1>{}); break;
            case 2: f(std::integral_constant<int, 2>{}); break;
            case 3: f(std::integral_constant<int, 3>{}); break;
            default: throw Error(IGAMG_EINVAL, "3D degree must be 1..3");
        }
    }
    // Calls f(op) with the operator view of level l in precision T.
    template <typename T, class F>
    void with_op(int l, F&& f) {
        Level& v = lv[l];
        if (kind == OP_STENCIL2D) {
            with_p([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                Stencil2D<P, T> op{v.coef<T>(), v.n, v.ncp};
                f(op);
            });
        } else if (kind == OP_KRON2D) {
            with_p([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                Kron2D<P, T> op{v.Kb<T>(), v.Mb<T>(), v.n, v.ncp};
                f(op);
            });
        } else {
            with_p3([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                Kron3D<P, T> op{v.Kb<T>(), v.Mb<T>(), v.n, v.ncp};
                f(op);
            });
        }
    }

    // Per-block sums written by residual(): one per 64-point block, or per
    // x-row on the 3D levels of the row kernels.
    long long residual_blocks(int l) const {
        const Level& v = lv[l];
        if (kind == OP_STENCIL2D) return (long long)v.ncol * (v.ncp / 64);
        if (kron_rows_available(l)) return (dim == 3) ? (long long)v.n * v.n : (long long)v.n;
        return (v.N + 63) / 64;
    }

    // out = b - A x (mode 0), A x (mode 1), Jacobi step (mode 2), z = D^{-1}(b - A x)
    // as float with per-block sums of z^2 in part (mode 3)
    // (sum-factorised levels: one workgroup per x-row, modes 0-2)
    template <typename T, typename Tout>
    void residual(int l, const T* bb, const T* x, Tout* out, int mode, double* part) {
        const long long nb = residual_blocks(l);
        with_op<T>(l, [&](auto op) {
            using Op = decltype(op);
            if constexpr (!Op::kColourOrder) {
                if (kron_rows_available(l)) {
                    if (mode > 2) throw Error(IGAMG_EINVAL, "residual mode 3 needs stored stencils");
                    const int n = lv[l].n;
                    if constexpr (is_kron3<Op>()) {
                        if (n < kResRollMinN || n > kResRollMaxN) {
                            hipLaunchKernelGGL((k_residual_row_kron<Op, Tout>), dim3((unsigned)nb),
                                               dim3(((n + 63) / 64) * 64), row_kron_lds_bytes(p, n, 2, sizeof(T)),
                                               stream, op, bb, x, out, mode, opt.omega, part);
                            check_launch();
                            return;
                        }
                        const unsigned grid = (unsigned)n * ((n + kResRollPlanes - 1) / kResRollPlanes);
                        hipLaunchKernelGGL((k_residual_roll_kron3<Op, Tout>), dim3(grid), dim3(((n + 63) / 64) * 64),
                                           res_roll_lds_bytes(p, n, sizeof(T)), stream, op, bb, x, out, mode,
                                           opt.omega, part);
                    } else {
                        hipLaunchKernelGGL((k_residual_row_kron<Op, Tout>), dim3((unsigned)nb),
                                           dim3(((n + 63) / 64) * 64), row_kron_lds_bytes(p, n, 2, sizeof(T)),
                                           stream, op, bb, x, out, mode, opt.omega, part);
                    }
                    check_launch();
                    return;
                }
            }
            hipLaunchKernelGGL((k_residual_sliced<Op, Tout>), dim3((unsigned)nb), dim3(64 * Op::NW), 0,
                               stream, op, bb, x, out, mode, opt.omega, lv[l].N, part);
        });
        check_launch();
    }

    // Bytes of level l's stored coefficients in a precision (0 for Kronecker operators).
    long long coef_bytes(int l, size_t elem) const {
        if (kind != OP_STENCIL2D) return 0;
        const long long W = 2 * p + 1;
        return (long long)lv[l].ncol * W * W * lv[l].ncp * (long long)elem;
    }
    static constexpr long long kCachedCoefBytes = 64LL << 20;

    template <typename T>
    void smooth(int l, const T* bb, T* x, int nsweeps) {
        Level& v = lv[l];
        for (int s = 0; s < nsweeps; ++s) {
            if (opt.smoother == IGAMG_SMOOTH_LEXGS) {
                with_op<T>(l, [&](auto op) {
                    using Op = decltype(op);
                    if constexpr (std::is_same_v<typename Op::Pt, Pt2>)
                        hipLaunchKernelGGL((k_lexgs_sweep<Op>), dim3(1), dim3(kLexThreads), 0, stream, op, bb, x);
                });
                check_launch();
                continue;
            }
            if (opt.smoother == IGAMG_SMOOTH_JACOBI) {
                residual<T, T>(l, bb, x, v.r<T>(), 2, nullptr);
                copy(v.r<T>(), x, v.N);
                continue;
            }
            mc_sweep<T>(l, bb, x);
        }
    }

    // Stored-stencil levels narrow enough for the LDS row store (and with at
    // most kRowThreads points per colour and row) sweep the p+1 colours of a
    // row class in one launch.
    // (the kernel addresses a level's coefficients with 32-bit byte offsets)
    bool row_sweeps(int l) const {
        return row_sweeps_available(l) && (l >= (int)row_pref.size() || row_pref[l] != 0);
    }
    // Sweep launches of level l in use: 0 one per colour, 1 one per row
    // class, 2 one per plane class (3D).
    int sweep_shape(int l) const {
        if (!row_sweeps(l)) return 0;
        return (l < (int)row_pref.size() && row_pref[l] == 2 && plane3_available(l)) ? 2 : 1;
    }
    // Sum-factorised 3D levels whose planes (with the waves' row buffers) fit
    // the plane-class kernel's LDS in FP64, one lane per point of a row.
    // (LDS for the planes in the sweeps' precision: FP64 solves, or FP32
    // V-cycles inside FP64 refinement)
    bool plane3_available(int l) const {
        const int elem = (opt.precision == IGAMG_FP64) ? 8 : 4;
        return kind == OP_KRON3D && kron_rows_available(l) && lv[l].n <= kPlane3MaxN &&
               plane3_lds_bytes(p, lv[l].n, elem) <= kPlane3MaxLds;
    }
    // The plane-class kernels and the 3D residual of the large levels take more
    // than the default dynamic LDS; the attribute is raised once per context,
    // before any launch or capture.
    void raise_kron3_lds() {
        if (kind != OP_KRON3D) return;
        auto raise = [](const void* f, int bytes) {
            IGAMG_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
        };
        with_p3([&](auto PC) {
            constexpr int P = decltype(PC)::value;
            using F = Kron3D<P, float>;
            using D = Kron3D<P, double>;
            raise(reinterpret_cast<const void*>(&k_gs_planeclass3<F>), kPlane3MaxLds);
            raise(reinterpret_cast<const void*>(&k_gs_planeclass3<D>), kPlane3MaxLds);
            const int roll = res_roll_lds_bytes(P, kResRollMaxN, sizeof(double));
            raise(reinterpret_cast<const void*>(&k_residual_roll_kron3<F, float>), roll);
            raise(reinterpret_cast<const void*>(&k_residual_roll_kron3<D, float>), roll);
            raise(reinterpret_cast<const void*>(&k_residual_roll_kron3<D, double>), roll);
        });
    }
    bool row_sweeps_available(int l) const {
        if (kind != OP_STENCIL2D) return kron_rows_available(l);
        // (the row kernel's register bound: p <= 4 in FP64, p <= 5 in FP32)
        const bool deg_ok = p <= 4 || (p == 5 && opt.precision == IGAMG_FP32_IR);
        return opt.row_sweeps && kind == OP_STENCIL2D && deg_ok && row_fits(p, lv[l].n) &&
               coef_bytes(l, sizeof(double)) < (1LL << 32);
    }
    // Sum-factorised levels of at most kRowKronMaxN unknowns per direction:
    // row-class sweeps and one-workgroup-per-row residuals.
    bool kron_rows_available(int l) const {
        return opt.row_sweeps && (kind == OP_KRON3D || kind == OP_KRON2D) && lv[l].n <= kRowKronMaxN;
    }
    // One multicolour Gauss-Seidel sweep of level l (multi-block launches).
    // Returns the number of launches; *bytes (when given) receives the
    // algorithmic bytes: per updated point its coefficients, b, and x read
    // and written.
    template <typename T>
    int mc_sweep(int l, const T* bb, T* x, double* bytes = nullptr) {
        Level& v = lv[l];
        // coefficients of levels up to kCachedCoefBytes are re-read from
        // cache by the next sweep; larger levels stream them
        const bool stream_coef = coef_bytes(l, sizeof(T)) > kCachedCoefBytes;
        const int W = 2 * p + 1;
        const long long S = (dim == 2) ? W * W : (long long)W * W * W;
        const double per_point = (kind == OP_STENCIL2D ? (double)S : 0.0) * sizeof(T) + 3.0 * sizeof(T);
        int launches = 0;
        with_op<T>(l, [&](auto op) {
            using Op = decltype(op);
            if constexpr (!Op::kColourOrder) {
                if constexpr (std::is_same_v<typename Op::Pt, Pt3>) {
                    if (sweep_shape(l) == 2) {
                        const int P1 = p + 1;
                        const size_t lds = plane3_lds_bytes(p, v.n, sizeof(T));
                        const int th = 64 * plane3_waves(p, v.n);
                        for (int ck = 0; ck < P1; ++ck) {
                            const int nk = (v.n - ck + p) / P1;
                            if (nk <= 0) continue;
                            hipLaunchKernelGGL((k_gs_planeclass3<Op>), dim3(nk), dim3(th), lds, stream, op, bb,
                                               x, ck);
                            ++launches;
                            if (bytes)
                                for (int c = P1 * P1 * ck; c < P1 * P1 * (ck + 1); ++c)
                                    *bytes += colour_size_host(v.n, p, dim, c) * per_point;
                        }
                        return;
                    }
                }
                if (row_sweeps(l)) {
                    const int P1 = p + 1;
                    const size_t lds = row_kron_lds_bytes(p, v.n, 3, sizeof(T));
                    const int th = ((v.n + 63) / 64) * 64;
                    for (int ck = 0; ck < (dim == 3 ? P1 : 1); ++ck)
                        for (int cj = 0; cj < P1; ++cj) {
                            const int nj = (v.n - cj + p) / P1, nk = (dim == 3) ? (v.n - ck + p) / P1 : 1;
                            if (nj <= 0 || nk <= 0) continue;
                            hipLaunchKernelGGL((k_gs_rowclass_kron<Op>), dim3(nj * nk), dim3(th), lds, stream, op,
                                               bb, x, cj, ck);
                            ++launches;
                            if (bytes)
                                for (int ci = 0; ci < P1; ++ci)
                                    *bytes += colour_size_host(v.n, p, dim, ci + P1 * (cj + P1 * ck)) * per_point;
                        }
                    return;
                }
            }
            if constexpr (Op::kColourOrder) {
                if constexpr (row_kernel_ok<Op>()) {
                    if (row_sweeps(l)) {
                        const int th = row_threads(p, v.n);
                        for (int r = 0; r <= p; ++r) {
                            const int nj = (v.n - r + p) / (p + 1);
                            if (nj <= 0) continue;
                            if (stream_coef)
                                hipLaunchKernelGGL((k_gs_rowclass<Op, true>), dim3(nj), dim3(th), 0, stream,
                                                   op, bb, x, r);
                            else
                                hipLaunchKernelGGL((k_gs_rowclass<Op, false>), dim3(nj), dim3(th), 0, stream,
                                                   op, bb, x, r);
                            ++launches;
                            if (bytes)
                                for (int s = 0; s <= p; ++s)
                                    *bytes += colour_size_host(v.n, p, dim, s + (p + 1) * r) * per_point;
                        }
                        return;
                    }
                }
            }
            for (int c = 0; c < v.ncol; ++c) {
                int cs = colour_size_host(v.n, p, dim, c);
                if (cs == 0) continue;
                if (stream_coef)
                    hipLaunchKernelGGL((k_gs_colour_sliced<Op, true>), dim3((cs + 63) / 64),
                                       dim3(64 * Op::NW), 0, stream, op, bb, x, c);
                else
                    hipLaunchKernelGGL((k_gs_colour_sliced<Op, false>), dim3((cs + 63) / 64),
                                       dim3(64 * Op::NW), 0, stream, op, bb, x, c);
                ++launches;
                if (bytes) *bytes += cs * per_point;
            }
        });
        check_launch();
        return launches;
    }

    // bc = R rf; xc (optional) zeroed in the same pass
    template <typename T>
    void restrict_(int l, const T* rf, T* bc, T* xc = nullptr) {
        Level& f = lv[l];
        Level& c = lv[l - 1];
        if (dim == 2)
            with_p([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                hipLaunchKernelGGL((k_restrict2d<P, T>), dim3(grid_for(c.N)), dim3(kBlock), 0, stream, rf,
                                   f.n, bc, c.n, f.r_start, f.rw<T>(), f.RW, xc);
            });
        else
            with_p3([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                hipLaunchKernelGGL((k_restrict3d<P, T>), dim3(grid_for(c.N)), dim3(kBlock), 0, stream, rf,
                                   f.n, bc, c.n, f.r_start, f.rw<T>(), f.RW, xc);
            });
        check_launch();
    }

    // Work items (64-point chunks x slices) of the largest colour of level l.
    int colour_items(int l) const {
        int mx = 0;
        for (int c = 0; c < lv[l].ncol; ++c) mx = std::max(mx, colour_size_host(lv[l].n, p, dim, c));
        return ((mx + 63) / 64) * (2 * p + 1);
    }
    std::string tune_key() const {
        hipDeviceProp_t prop;
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::string arch = "?";
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
        return arch + "/" + std::to_string(geom) + "/" + std::to_string(opt.pde) + "/" + std::to_string(p) + "/" +
               std::to_string(lv[L].n_el) + "/" + std::to_string(opt.precision);
    }
    // Launch-shape defaults: row-class sweeps wherever they apply; the learned
    // step with 28 x 28 tiles (512 threads) on levels of 384 unknowns per
    // direction and more, 12 x 12 tiles below (the faster of the two measured
    // on the 1024^2 annulus hierarchy, p = 3).
    void default_shapes() {
        row_pref.assign(L + 1, 1);
        for (int l = 0; l <= L; ++l)
            if (plane3_available(l)) row_pref[l] = 2;
        learned_kern.assign(L + 1, 12);
        for (int l = 0; l <= L; ++l)
            if (lv[l].n >= 384) learned_kern[l] = 28;
    }
    void apply_choice(const TuneChoice& c) {
        opt.tail_items = c.tail_items;
        if ((int)c.row.size() == L + 1) row_pref = c.row;
        if ((int)c.learned.size() == L + 1) learned_kern = c.learned;
        tuned_ms = c.vcycle_ms;
        graph_method = -1;
    }
    // Takes the cached choice of this problem and precision, if there is one.
    bool apply_cached_choice() {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(tune_key());
        if (it == g_tune_cache.end()) return false;
        apply_choice(it->second);
        return true;
    }
    void choose_tail() {
        tail_top = 0;
        if (opt.smoother != IGAMG_SMOOTH_MCGS) return;  // the single-workgroup kernel sweeps colours
        if (opt.tail_items < 0) {
            tail_auto = true;
            if (!apply_cached_choice()) opt.tail_items = 32;
        }
        if (opt.tail_items <= 0) return;
        const int limit = (opt.precision == IGAMG_FP64) ? tail_limit<double>() : tail_limit<float>();
        for (int l = 1; l <= limit; ++l) {
            if (colour_items(l) > opt.tail_items) break;
            tail_top = l;
        }
    }
    // Finest level whose iterates, with those of all coarser levels, fit the
    // single-workgroup kernel's LDS store in precision T.
    template <typename T>
    int tail_limit() {
        long long used = 0;
        int top = 0;
        for (int l = 0; l <= L && l < kTailMaxLevels; ++l) {
            used += tail_level_size<T>(l);
            if (used + kTailPadVals > tail_capacity<T>() || !tail_level_ok<T>(l)) break;
            top = l;
        }
        return top;
    }
    // The prefetching tail variant (FP32 stored stencils) needs the records of
    // every level it smooths, which exist where a colour fits the block;
    // sum-factorised levels need rows of at most one wave.
    template <typename T>
    bool tail_level_ok(int l) {
        if (kind != OP_STENCIL2D && lv[l].n > kTailKronMaxN) return false;  // one lane per point of a row
        bool ok = true;
        with_op<T>(l, [&](auto opl) {
            if constexpr (tail_prefetch<decltype(opl)>()) ok = (l == 0) || lv[l].rec32 != nullptr;
        });
        return ok;
    }
    // LDS values that level l takes in the single-workgroup kernel: the padded
    // iterate for stored 2D stencils; the natural iterate plus (l >= 1) the two
    // 1D bands for sum-factorised operators.
    template <typename T>
    long long tail_level_size(int l) {
        long long sz = lv[l].N + (l >= 1 ? 2LL * lv[l].n * (2 * p + 1) : 0);
        with_op<T>(l, [&](auto opl) {
            if constexpr (decltype(opl)::kColourOrder) sz = tl_size(p, tl_vw(sizeof(T)), lv[l].n);
        });
        return sz;
    }

    // Arguments of the single-workgroup V-cycle on levels 0..tail_top.
    template <class Op>
    TailArgs<Op> tail_args(const typename Op::T* bt, typename Op::T* xt) {
        using T = typename Op::T;
        TailArgs<Op> a{};
        a.top = tail_top;
        a.nu1 = opt.nu1;
        a.nu2 = opt.nu2;
        a.mu = opt.mu;
        a.n0 = n0;
        a.Ainv = Ainv0;
        long long off = 0;
        for (int l = 0; l <= tail_top; ++l) {
            with_op<T>(l, [&](auto opl) {
                if constexpr (std::is_same_v<decltype(opl), Op>) a.op[l] = opl;
            });
            a.N[l] = lv[l].N;
            if constexpr (Op::kColourOrder) {
                a.xoff[l] = (int)off;  // a multiple of the vector width
            } else {
                a.boff[l] = (int)off;  // bands K, M (levels >= 1), then the iterate
                a.xoff[l] = (int)(off + (l >= 1 ? 2LL * lv[l].n * (2 * p + 1) : 0));
            }
            off += tail_level_size<T>(l);

            a.x[l] = (l == tail_top) ? xt : lv[l].x<T>();
            a.b[l] = (l == tail_top) ? (T*)bt : lv[l].b<T>();
            a.r[l] = lv[l].r<T>();
            if constexpr (std::is_same_v<T, float>) a.rec[l] = lv[l].rec32;
            {
                int mx = 0;
                for (int c = 0; c < lv[l].ncol; ++c) mx = std::max(mx, colour_size_host(lv[l].n, p, dim, c));
                a.act[l] = std::max(1, (mx + 63) / 64);
            }
            if (!tail_level_ok<T>(l)) throw Error(IGAMG_EINVAL, "tail level without coefficient records");
            if (l >= 1) {
                a.rs[l] = lv[l].r_start;
                a.rw[l] = lv[l].rw<T>();
                a.ps[l] = lv[l].p_start;
                a.pw[l] = lv[l].pw<T>();
                a.RW[l] = lv[l].RW;
                a.PW[l] = lv[l].PW;
            }
        }
        if (tail_top >= kTailMaxLevels || off + kTailPadVals > tail_capacity<T>())
            throw Error(IGAMG_EINVAL, "levels 0..tail_top do not fit the single-workgroup kernel");
        return a;
    }

    // V-cycle on levels 0..tail_top by one workgroup.
    template <typename T>
    void tail(const T* bt, T* xt) {
        with_op<T>(0, [&](auto op0) {
            using Op = decltype(op0);
            TailArgs<Op> a = tail_args<Op>(bt, xt);
            hipLaunchKernelGGL((k_vcycle_tail<Op>), dim3(1), dim3(tail_threads<Op>()), 0, stream, a);
        });
        check_launch();
    }
    template <typename T>
    void prolong_(int l, const T* ec, T* xf) {
        Level& f = lv[l];
        Level& c = lv[l - 1];
        if (dim == 2)
            with_p([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                hipLaunchKernelGGL((k_prolong2d<P, T>), dim3(grid_for(f.N)), dim3(kBlock), 0, stream, ec,
                                   c.n, xf, f.n, f.p_start, f.pw<T>(), f.PW);
            });
        else
            with_p3([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                hipLaunchKernelGGL((k_prolong3d<P, T>), dim3(grid_for(f.N)), dim3(kBlock), 0, stream, ec,
                                   c.n, xf, f.n, f.p_start, f.pw<T>(), f.PW);
            });
        check_launch();
    }
    template <typename T>
    void coarse(const T* bb, T* x) {
        hipLaunchKernelGGL(k_coarse_solve<T>, dim3(1), dim3(kBlock), 0, stream, Ainv0, n0, bb, x);
        check_launch();
    }

    template <typename T> T* diag(int l) {
        if constexpr (std::is_same_v<T, double>) return diag64[l]; else return diag32[l];
    }
    bool use_learned(int l) const {
        return learned_on && l > tail_top && l < (int)nets.size() && nets[l].have && nets[l].on;
    }
    // Learned first pre-smoothing step on level l: x += sigma N_l(D^{-1} r / sigma).
    // The residual kernel writes z = D^{-1} r and per-block sums of z^2 directly;
    // when x is known to be zero (x_zero), r = b and the same z and sums come
    // from b and the stencil centres alone.
    template <typename T>
    void learned_step(int l, const T* bl, T* xl, bool x_zero = false) {
        Level& v = lv[l];
        bool done = false;
        if (x_zero)
            with_op<T>(l, [&](auto op) {
                using Op = decltype(op);
                if constexpr (Op::kColourOrder) {
                    hipLaunchKernelGGL((k_scaled_rhs<Op>), dim3((unsigned)residual_blocks(l)), dim3(64), 0,
                                       stream, op, bl, lz, partial);
                    done = true;
                }
            });
        if (!done) residual<T, float>(l, bl, xl, lz, 3, partial);
        hipLaunchKernelGGL(k_learned_sigma, dim3(1), dim3(kLSigmaThreads), 0, stream, partial,
                           (int)residual_blocks(l), v.N, scal + 2);
        LImage im{lz, v.n, v.n, v.n, 0, 0};
        learned_apply<T>(l, im, (const double*)(scal + 2), xl, nullptr);
    }

    // Inference launch of the network on one level image: x += sigma N(z / sigma)
    // (yout null) or yout = N(z).  The level's learned_kern selects the kernel: 0 the
    // 16 x 16 VALU / MFMA tile kernel, 12 / 28 the all-MFMA kernel with that
    // output tile (28: 512 threads, 29: tile 28 with 256 threads).
    template <typename T>
    void learned_apply(int l, const LImage& im, const double* sigma, T* xl, float* yout) {
        learned_apply_k<T>(learned_kern[l], nets[l], im, sigma, xl, yout);
    }
    template <typename T>
    void learned_apply_k(int kern_id, const Net& net, const LImage& im, const double* sigma, T* xl,
                         float* yout) {
        auto go = [&](auto kern, int tl, int nt) {
            const int tiles = (im.width + tl - 1) / tl;
            hipLaunchKernelGGL(kern, dim3(tiles * tiles), dim3(nt), 0, stream, im, (const float*)net.mf32,
                               (const uint16_t*)net.mfbf, sigma, xl, yout);
        };
        switch (kern_id) {
            case 12: go(k_learned_apply_mf<12, 256, T>, 12, 256); break;
            case 28: go(k_learned_apply_mf<28, 512, T>, 28, 512); break;
            case 29: go(k_learned_apply_mf<28, 256, T>, 28, 256); break;
            default: {
                const int tiles = (im.width + kLTile - 1) / kLTile;
                LearnedW W{net.wc, net.w2f, net.w2b};
                hipLaunchKernelGGL(k_learned_apply<T>, dim3(tiles * tiles), dim3(kLThreads), 0, stream, im, W,
                                   sigma, xl, yout);
            }
        }
        check_launch();
    }

    // Levels 0..tt of a cycle on level l-1 (l-1 <= tt): the single-workgroup
    // kernel when tt >= 1, else the coarse solve.
    template <typename T>
    void bottom(int tt, const T* bl, T* xl) {
        if (tt >= 1) {
            int save = tail_top;
            tail_top = tt;
            tail<T>(bl, xl);
            tail_top = save;
        } else {
            coarse<T>(bl, xl);
        }
    }
    // One mu-cycle (Algorithm 2, mu = opt.mu > 1) on a level l > tt: the
    // coarse cycle runs mu times on the same restricted residual, each call
    // after the first starting from the previous result.
    template <typename T>
    void mucycle(int l, int tt, const T* bl, T* xl) {
        if (use_learned(l)) {
            learned_step<T>(l, bl, xl);
            smooth<T>(l, bl, xl, opt.nu1 - 1);
        } else {
            smooth<T>(l, bl, xl, opt.nu1);
        }
        residual<T, T>(l, bl, xl, lv[l].r<T>(), 0, nullptr);
        restrict_<T>(l, lv[l].r<T>(), lv[l - 1].b<T>(), lv[l - 1].x<T>());
        for (int k = 0; k < opt.mu; ++k) {
            if (l - 1 > tt)
                mucycle<T>(l - 1, tt, lv[l - 1].b<T>(), lv[l - 1].x<T>());
            else
                bottom<T>(tt, lv[tt].b<T>(), lv[tt].x<T>());
        }
        prolong_<T>(l, lv[l - 1].x<T>(), xl);
        smooth<T>(l, bl, xl, opt.nu2);
    }

    // One V(nu1, nu2) cycle (Algorithm 2; the mu-cycle when opt.mu > 1) in
    // precision T starting on level `top` with right-hand side bt and iterate
    // xt (in place).  Levels above tail_top launch one kernel per step; levels
    // 0..min(top, tail_top) run in one single-workgroup kernel.  `rec`, when
    // given (V-cycles only), is called at the start of every level l >= 1
    // with (l, b_l, x_l).
    // xt_zero: the caller guarantees xt = 0 on entry (every coarser level
    // starts from zero anyway).
    template <typename T, class Rec = std::nullptr_t>
    void vcycle_from(int top, const T* bt, T* xt, Rec rec = nullptr, bool xt_zero = false) {
        if (top == 0) {
            coarse<T>(bt, xt);
            return;
        }
        const int tt = std::min({tail_top, top, tail_limit<T>()});
        if (opt.mu > 1) {
            if constexpr (!std::is_same_v<Rec, std::nullptr_t>)
                throw Error(IGAMG_EINVAL, "recording levels needs mu = 1");
            if (top <= tt)
                bottom<T>(tt, bt, xt);
            else
                mucycle<T>(top, tt, bt, xt);
            return;
        }
        for (int l = top; l > tt; --l) {
            const T* bl = (l == top) ? bt : lv[l].b<T>();
            T* xl = (l == top) ? xt : lv[l].x<T>();
            if constexpr (!std::is_same_v<Rec, std::nullptr_t>) rec(l, bl, xl);
            if (use_learned(l)) {
                learned_step<T>(l, bl, xl, l < top || xt_zero);
                smooth<T>(l, bl, xl, opt.nu1 - 1);
            } else {
                smooth<T>(l, bl, xl, opt.nu1);
            }
            residual<T, T>(l, bl, xl, lv[l].r<T>(), 0, nullptr);
            restrict_<T>(l, lv[l].r<T>(), lv[l - 1].b<T>(), lv[l - 1].x<T>());
        }
        bottom<T>(tt, (tt == top) ? bt : lv[tt].b<T>(), (tt == top) ? xt : lv[tt].x<T>());
        for (int l = tt + 1; l <= top; ++l) {
            const T* bl = (l == top) ? bt : lv[l].b<T>();
            T* xl = (l == top) ? xt : lv[l].x<T>();
            prolong_<T>(l, lv[l - 1].x<T>(), xl);
            smooth<T>(l, bl, xl, opt.nu2);
        }
    }
    template <typename T>
    void vcycle(const T* bL, T* xL) { vcycle_from<T>(L, bL, xL); }

    // The fixed-point map G of eq. (7) on the finest level, in place.
    void G(double* x) {
        if (opt.precision == IGAMG_FP64) {
            vcycle<double>(b, x);
            return;
        }
        Level& f = lv[L];
        residual<double, float>(L, b, x, f.b32, 0, nullptr);  // round32(b - A x)
        fill(f.x32, f.N);
        vcycle_from<float>(L, f.b32, f.x32, nullptr, true);
        hipLaunchKernelGGL(k_add_f32_to_f64, dim3(grid_for(f.N)), dim3(kBlock), 0, stream, f.x32, x,
                           f.N);
        check_launch();
    }

    // scal[0] = ||b - A x|| / ||b|| (device); no host synchronisation.
    void resnorm_async(const double* x) {
        residual<double, double>(L, b, x, lv[L].r64, 0, partial);
        long long nb = residual_blocks(L);
        hipLaunchKernelGGL(k_finalize_norm, dim3(1), dim3(kBlock), 0, stream, partial, (int)nb, 1.0,
                           (const double*)(scal + 1), scal);
        check_launch();
    }

    // Stores ||b|| (1 for a zero right-hand side) where the residual kernels read it.
    void set_bnorm(double v) {
        bnorm = v;
        host_scal[1] = v > 0.0 ? v : 1.0;
        IGAMG_HIP(hipMemcpyAsync(scal + 1, host_scal + 1, sizeof(double), hipMemcpyHostToDevice, stream));
        sync();
    }

    // Relative residual and extrapolation status of the last restart cycle.
    double read_cycle(ExtrapCoeffs& c) {
        IGAMG_HIP(hipMemcpyAsync(host_scal, scal, sizeof(double), hipMemcpyDeviceToHost, stream));
        IGAMG_HIP(hipMemcpyAsync(host_coeffs, coeffs, sizeof(ExtrapCoeffs), hipMemcpyDeviceToHost, stream));
        IGAMG_HIP(hipStreamSynchronize(stream));
        c = *host_coeffs;
        last_coeffs = c;
        have_coeffs = true;
        return host_scal[0];
    }

    void ensure_iterates(int q) {
        while ((int)S.size() < q + 2) S.push_back(alloc<double>(lv[L].N));
        if (!ckpt) ckpt = alloc<double>(lv[L].N);
        int ncols = q + 1;
        long long leaves = (lv[L].N + kQrRows - 1) / kQrRows;
        size_t need = (size_t)leaves * ncols * ncols;
        if (need > Rcap) {
            release(Rbuf[0]);
            release(Rbuf[1]);
            Rbuf[0] = alloc<double>(need);
            Rbuf[1] = alloc<double>(need);
            Rcap = need;
        }
    }

    // Tall-skinny QR tree of Delta S from iterates it[0..q+1] and the small
    // solve; result in coeffs (device).
    void extrap_coeffs_async(const IterPtrs& it, int q, int method) {
        tsqr_coeffs_async(stream, it, q, lv[L].N, method, Rbuf[0], Rbuf[1], coeffs);
    }

    IterPtrs iter_ptrs(int q) {
        IterPtrs it{};
        for (int j = 0; j <= q + 1; ++j) it.s[j] = S[j];
        return it;
    }

    // One restart cycle (Algorithm 5 body) on the iterate buffers: S[0] holds
    // s_0 on entry and t on exit (s_0 again if the coefficients are not
    // finite), ckpt receives s_0; the residual norm of S[0] goes to scal[0]
    // (unless with_resnorm is false).
    void restart_cycle(int method, int q, bool with_resnorm = true) {
        long long N = lv[L].N;
        for (int j = 0; j <= q; ++j) {
            copy(S[j], S[j + 1], N);
            G(S[j + 1]);
        }
        IterPtrs it = iter_ptrs(q);
        extrap_coeffs_async(it, q, method);
        hipLaunchKernelGGL(k_extrap_combine, dim3(grid_for(N)), dim3(kBlock), 0, stream, it, q, N,
                           (const ExtrapCoeffs*)coeffs, S[0], ckpt);
        check_launch();
        if (with_resnorm) resnorm_async(S[0]);
    }

    // Plain multigrid step on S[0]: one application of G and the residual norm;
    // ckpt receives the iterate it starts from.
    void plain_cycle() {
        copy(S[0], ckpt, lv[L].N);
        G(S[0]);
        resnorm_async(S[0]);
    }

    void run_restart_cycle(int method, int q, bool with_resnorm = true) {
        if (method == IGAMG_EXTRAP_NONE) with_resnorm = true;
        if (!opt.use_graphs) {
            if (method == IGAMG_EXTRAP_NONE)
                plain_cycle();
            else
                restart_cycle(method, q, with_resnorm);
            return;
        }
        if (!graph_exec || graph_method != method || graph_q != q || graph_resnorm != with_resnorm) {
            if (graph_exec) {
                (void)hipGraphExecDestroy(graph_exec);
                graph_exec = nullptr;
            }
            if (graph) {
                (void)hipGraphDestroy(graph);
                graph = nullptr;
            }
            IGAMG_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            try {
                if (method == IGAMG_EXTRAP_NONE)
                    plain_cycle();
                else
                    restart_cycle(method, q, with_resnorm);
            } catch (...) {
                hipGraph_t g;
                (void)hipStreamEndCapture(stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            IGAMG_HIP(hipStreamEndCapture(stream, &graph));
            IGAMG_HIP(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
            graph_method = method;
            graph_q = q;
            graph_resnorm = with_resnorm;
        }
        IGAMG_HIP(hipGraphLaunch(graph_exec, stream));
    }

    double read_scal() {
        IGAMG_HIP(hipMemcpyAsync(host_scal, scal, sizeof(double), hipMemcpyDeviceToHost, stream));
        IGAMG_HIP(hipStreamSynchronize(stream));
        return host_scal[0];
    }
    ExtrapCoeffs read_coeffs() {
        IGAMG_HIP(hipMemcpyAsync(host_coeffs, coeffs, sizeof(ExtrapCoeffs), hipMemcpyDeviceToHost, stream));
        IGAMG_HIP(hipStreamSynchronize(stream));
        last_coeffs = *host_coeffs;
        have_coeffs = true;
        return *host_coeffs;
    }
    void sync() { IGAMG_HIP(hipStreamSynchronize(stream)); }

    double vector_norm(const double* v, long long N) {
        unsigned nb = std::min<long long>(grid_for(N), 1024);
        hipLaunchKernelGGL(k_sumsq<double>, dim3(nb), dim3(kBlock), 0, stream, v, N, partial);
        check_launch();
        hipLaunchKernelGGL(k_finalize_norm, dim3(1), dim3(kBlock), 0, stream, partial, (int)nb, 1.0,
                           (const double*)nullptr, scal);
        check_launch();
        return read_scal();
    }

    // nsweeps multicolour sweeps of level l captured as one HIP graph (the form
    // in which a solve runs them), replayed once to warm up and once between
    // two events: avg = elapsed / launches.
    template <typename T>
    void profile_smoother_t(int l, int nsweeps, double* avg_ms, double* bytes, int* launches) {
        Level& v = lv[l];
        T* x = v.x<T>();
        T* bb = v.b<T>();
        fill(x, v.N);
        hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(v.N)), dim3(kBlock), 0, stream, bb, (T)1, v.N);
        check_launch();
        int total = 0;
        double tot_bytes = 0.0;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        IGAMG_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
            for (int sw = 0; sw < nsweeps; ++sw) total += mc_sweep<T>(l, bb, x, &tot_bytes);
        } catch (...) {
            (void)hipStreamEndCapture(stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        IGAMG_HIP(hipStreamEndCapture(stream, &g));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t err = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (err == hipSuccess) err = hipEventCreate(&e0);
        if (err == hipSuccess) err = hipEventCreate(&e1);
        if (err == hipSuccess) err = hipGraphLaunch(ge, stream);  // warm-up
        if (err == hipSuccess) err = hipEventRecord(e0, stream);
        if (err == hipSuccess) err = hipGraphLaunch(ge, stream);
        if (err == hipSuccess) err = hipEventRecord(e1, stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (ge) (void)hipGraphExecDestroy(ge);
        (void)hipGraphDestroy(g);
        if (err != hipSuccess) throw Error(IGAMG_EHIP, std::string("profile: ") + hipGetErrorString(err));
        *avg_ms = total ? ms / total : 0.0;
        *bytes = total ? tot_bytes / total : 0.0;
        *launches = total;
    }
    void profile_smoother(int l, int precision, int nsweeps, double* avg_ms, double* bytes,
                          int* launches) {
        if (precision == IGAMG_FP64)
            profile_smoother_t<double>(l, nsweeps, avg_ms, bytes, launches);
        else
            profile_smoother_t<float>(l, nsweeps, avg_ms, bytes, launches);
    }

    // ---- learned smoother support
    void setup_diag();
    void ensure_net(int l);
    double level_resnorm(int l, const double* f, const double* x, double fnorm);
    int level_solve(int l, const double* f, double* u, double tol, int maxit);
    void train(const igamg_train_options& o, igamg_train_report& rep);
    double measure_rho(int vcycles, bool learned);
    double measure_rho_level(int l, const double* f, int vcycles, bool learned);

    void autotune(int* best_items, double* best_ms, bool tune_learned = true);
    void precond_apply(int precond, int q, const double* v, double* z);
    void fgmres(double tol, int max_iters, int m, int precond, int q, double* x, igamg_stats& st);

    void setup(const igamg_geometry& g, int degree, int levels);
    void setup_levels(int n_el, int levels);
    void setup_kron();
    void setup_annulus();
    void setup_coarse();
    void setup_kron_stencils();
    void setup_records();
    void set_rhs_field(const double* modes, int n_modes);
};

// ---------------------------------------------------------------------------
// setup

void igamg_ctx::setup_levels(int n_el, int levels) {
    if (opt.n_el_coarsest <= 0) {
        int m = n_el;
        while (m > 7 && m % 2 == 0) m /= 2;
        while (m < 4 && m > 0) m *= 2;
        if (m < 4 || m > 7 || n_el % m) throw Error(IGAMG_EINVAL, "n_el is not m 2^k with m in 4..7");
        opt.n_el_coarsest = m;
    }
    int nc0 = opt.n_el_coarsest;
    if (nc0 < 1 || n_el < nc0 || n_el % nc0)
        throw Error(IGAMG_EINVAL, "n_el must be n_el_coarsest * 2^k");
    int k = 0;
    for (int m = n_el / nc0; m > 1; m /= 2) {
        if (m % 2) throw Error(IGAMG_EINVAL, "n_el must be n_el_coarsest * 2^k");
        ++k;
    }
    int nlev = k + 1;
    if (levels > 0) {
        if (levels > nlev) throw Error(IGAMG_EINVAL, "too many levels for this grid");
        nlev = levels;
    }
    L = nlev - 1;
    {
        long long nc = (n_el >> L) + p - 2, N0 = nc;
        for (int d = 1; d < dim; ++d) N0 *= nc;
        if (N0 > 4096) throw Error(IGAMG_EINVAL, "coarsest level too large for the dense direct solve");
    }
    lv.resize(nlev);
    for (int l = 0; l <= L; ++l) {
        Level& v = lv[l];
        v.n_el = n_el >> (L - l);
        v.n = v.n_el + p - 2;
        if (v.n < 1) throw Error(IGAMG_EINVAL, "level with no interior unknowns");
        v.N = 1;
        for (int d = 0; d < dim; ++d) v.N *= v.n;
        v.ncol = 1;
        for (int d = 0; d < dim; ++d) v.ncol *= (p + 1);
        int mx = 0;
        for (int c = 0; c < v.ncol; ++c) mx = std::max(mx, colour_size_host(v.n, p, dim, c));
        v.ncp = ((mx + kBlock - 1) / kBlock) * kBlock;
    }
    // transfer tables between l-1 and l by Boehm knot insertion
    for (int l = 1; l <= L; ++l) {
        Prolong1D P1 = prolongation_boehm(lv[l - 1].n_el, p);
        TransferTables T = transfer_tables(P1);
        if (T.nf != lv[l].n || T.nc != lv[l - 1].n) throw Error(IGAMG_EINVAL, "transfer size mismatch");
        Level& v = lv[l];
        v.RW = T.RW;
        v.PW = T.PW;
        // the transfer kernels unroll their windows to these bounds
        if (v.RW > restrict_bound(p) || v.PW > prolong_bound(p))
            throw Error(IGAMG_EINVAL, "transfer window wider than the knot-insertion bound");
        v.r_start = upload(T.r_start);
        v.p_start = upload(T.p_start);
        v.r_w64 = upload(T.r_w);
        v.p_w64 = upload(T.p_w);
        std::vector<float> rw32(T.r_w.begin(), T.r_w.end()), pw32(T.p_w.begin(), T.p_w.end());
        v.r_w32 = upload(rw32);
        v.p_w32 = upload(pw32);
    }
}

void igamg_ctx::setup_kron() {
    // finest 1D bands by quadrature, coarser ones by the 1D Galerkin product
    Band1D K, M;
    stiffness_mass_bands(lv[L].n_el, p, K, M);
    lv[L].Kh = K;
    lv[L].Mh = M;
    for (int l = L; l >= 1; --l) {
        Prolong1D P1 = prolongation_boehm(lv[l - 1].n_el, p);
        TransferTables T = transfer_tables(P1);
        lv[l - 1].Kh = galerkin_band(lv[l].Kh, T, p);
        lv[l - 1].Mh = galerkin_band(lv[l].Mh, T, p);
    }
    for (int l = 0; l <= L; ++l) {
        Level& v = lv[l];
        v.K64 = upload(v.Kh.v);
        v.M64 = upload(v.Mh.v);
        std::vector<float> k32(v.Kh.v.begin(), v.Kh.v.end()), m32(v.Mh.v.begin(), v.Mh.v.end());
        v.K32 = upload(k32);
        v.M32 = upload(m32);
    }
}

void igamg_ctx::setup_annulus() {
    const int W = 2 * p + 1, Sn = W * W;
    Level& f = lv[L];
    nq = p + 1;
    ElementTables E = element_tables(f.n_el, p, nq);
    tabV = upload(E.V);
    tabD = upload(E.D);
    tabPts = upload(E.pts);
    tabWts = upload(E.wts);
    const int NQ = f.n_el * nq;
    long long nqp = (long long)NQ * NQ;
    GeomQP G{};
    G.D11 = alloc<double>(nqp);
    G.D12 = alloc<double>(nqp);
    G.D22 = alloc<double>(nqp);
    G.wdet = alloc<double>(nqp);
    G.X = alloc<double>(nqp);
    G.Y = alloc<double>(nqp);
    if (opt.pde != IGAMG_PDE_POISSON) {
        G.Bx = alloc<double>(nqp);
        G.By = alloc<double>(nqp);
        G.Cw = alloc<double>(nqp);
    }
    hipLaunchKernelGGL(k_geometry_qp, dim3(grid_for(nqp)), dim3(kBlock), 0, stream, geom_params(), NQ,
                       tabPts, tabWts, G);
    check_launch();
    std::vector<double*> stage(L + 1, nullptr);
    stage[L] = alloc<double>((size_t)f.N * Sn);
    with_p([&](auto PC) {
        constexpr int P = decltype(PC)::value;
        hipLaunchKernelGGL(k_assemble_stencil<P>, dim3(grid_for(f.N * Sn)), dim3(kBlock), 0, stream,
                           f.n_el, nq, tabV, tabD, G, stage[L]);
    });
    check_launch();
    for (double* a : {G.D11, G.D12, G.D22, G.wdet, G.X, G.Y, G.Bx, G.By, G.Cw})
        if (a) release(a);
    // the Poisson operator is symmetric (Section 2, eq. (2)): make every level
    // exactly so (its assembly and the Galerkin products give it up to
    // rounding); the coarsest Cholesky factor then sees a symmetric matrix
    const bool sym = opt.pde == IGAMG_PDE_POISSON;
    auto symmetrize = [&](int l) {
        if (!sym) return;
        const long long cnt = lv[l].N * (long long)(p * W + p);
        with_p([&](auto PC) {
            constexpr int P = decltype(PC)::value;
            hipLaunchKernelGGL(k_symmetrize_stencil<P>, dim3(grid_for(cnt)), dim3(kBlock), 0, stream, stage[l],
                               lv[l].n);
        });
        check_launch();
        lv[l].sym = true;
    };
    symmetrize(L);
    // Galerkin coarse operators, separable: x pass then y pass
    for (int l = L; l >= 1; --l) {
        Level& fl = lv[l];
        Level& cl = lv[l - 1];
        double* Tm = alloc<double>((size_t)cl.n * fl.n * Sn);
        stage[l - 1] = alloc<double>((size_t)cl.N * Sn);
        with_p([&](auto PC) {
            constexpr int P = decltype(PC)::value;
            hipLaunchKernelGGL(k_rap_x<P>, dim3(grid_for((long long)cl.n * fl.n * Sn)), dim3(kBlock), 0,
                               stream, stage[l], fl.n, cl.n, fl.r_start, fl.r_w64, fl.RW, Tm);
            hipLaunchKernelGGL(k_rap_y<P>, dim3(grid_for(cl.N * Sn)), dim3(kBlock), 0, stream, Tm, fl.n,
                               cl.n, fl.r_start, fl.r_w64, fl.RW, stage[l - 1]);
        });
        check_launch();
        release(Tm);
        symmetrize(l - 1);
    }
    for (int l = 0; l <= L; ++l) {
        Level& v = lv[l];
        size_t cnt = (size_t)v.ncol * Sn * v.ncp;
        v.coef64 = alloc<double>(cnt);
        v.coef32 = alloc<float>(cnt);
        fill(v.coef64, (long long)cnt);
        fill(v.coef32, (long long)cnt);
        with_p([&](auto PC) {
            constexpr int P = decltype(PC)::value;
            hipLaunchKernelGGL(k_to_colour_blocked<P>, dim3(grid_for(v.N * Sn)), dim3(kBlock), 0, stream,
                               stage[l], v.n, v.ncp, v.coef64, v.coef32);
        });
        check_launch();
    }
    // coarsest dense matrix from the natural stencil rows
    Level& c = lv[0];
    std::vector<double> st((size_t)c.N * Sn);
    IGAMG_HIP(hipMemcpyAsync(st.data(), stage[0], st.size() * sizeof(double), hipMemcpyDeviceToHost,
                             stream));
    sync();
    for (int l = 0; l <= L; ++l) release(stage[l]);
    n0 = (int)c.N;
    std::vector<double> A((size_t)n0 * n0, 0.0);
    for (int I = 0; I < n0; ++I) {
        int j = I / c.n, i = I % c.n;
        for (int o = 0; o < Sn; ++o) {
            int i2 = i + o % W - p, j2 = j + o / W - p;
            if (i2 < 0 || i2 >= c.n || j2 < 0 || j2 >= c.n) continue;
            A[(size_t)I * n0 + i2 + c.n * j2] = st[(size_t)I * Sn + o];
        }
    }
    // nonsymmetric operators: LU with partial pivoting; Poisson: Cholesky
    std::vector<double> inv;
    if (coarse_inverse(std::move(A), n0, sym, inv) != 0)
        throw Error(IGAMG_ENOTSPD, sym ? "coarsest operator is not SPD" : "coarsest operator is singular");
    Ainv0 = upload(inv);
}

void igamg_ctx::setup_coarse() {
    // Kronecker coarsest operator expanded to a dense matrix
    Level& c = lv[0];
    n0 = (int)c.N;
    std::vector<double> A((size_t)n0 * n0, 0.0);
    const Band1D &K = c.Kh, &M = c.Mh;
    int n = c.n;
    for (int I = 0; I < n0; ++I) {
        int i = I % n, j = (I / n) % n, k = (dim == 3) ? I / (n * n) : 0;
        for (int J = 0; J < n0; ++J) {
            int i2 = J % n, j2 = (J / n) % n, k2 = (dim == 3) ? J / (n * n) : 0;
            int di = i2 - i, dj = j2 - j, dk = k2 - k;
            if (std::abs(di) > p || std::abs(dj) > p || std::abs(dk) > p) continue;
            double v;
            if (dim == 2)
                v = K.at(i, di) * M.at(j, dj) + M.at(i, di) * K.at(j, dj);
            else
                v = K.at(i, di) * M.at(j, dj) * M.at(k, dk) + M.at(i, di) * K.at(j, dj) * M.at(k, dk) +
                    M.at(i, di) * M.at(j, dj) * K.at(k, dk);
            A[(size_t)I * n0 + J] = v;
        }
    }
    std::vector<double> inv;
    if (coarse_inverse(std::move(A), n0, true, inv) != 0)
        throw Error(IGAMG_ENOTSPD, "coarsest operator is not SPD");
    Ainv0 = upload(inv);
}

// Per-point FP32 coefficient records of the levels whose colours fit the
// prefetching single-workgroup kernel's block (one point per thread).
void igamg_ctx::setup_records() {
    for (int l = 1; l <= L; ++l) {
        Level& v = lv[l];
        int mx = 0;
        for (int c = 0; c < v.ncol; ++c) mx = std::max(mx, colour_size_host(v.n, p, dim, c));
        if (mx > pf_threads(p)) continue;
        const long long cnt = (long long)v.ncol * v.ncp * rec_len(p);
        v.rec32 = alloc<float>(cnt);
        with_p([&](auto PC) {
            constexpr int P = decltype(PC)::value;
            hipLaunchKernelGGL(k_to_records<P>, dim3(grid_for(cnt)), dim3(kBlock), 0, stream,
                               (const float*)v.coef32, v.ncp, v.ncol, v.rec32);
        });
        check_launch();
    }
}

// Unit square with stored stencils: every level's (2p+1)^2 rows written out
// from its Kronecker factors (the same operator, one operator type for all 2D
// problems of a batch).
void igamg_ctx::setup_kron_stencils() {
    const int W = 2 * p + 1, Sn = W * W;
    for (int l = 0; l <= L; ++l) {
        Level& v = lv[l];
        size_t cnt = (size_t)v.ncol * Sn * v.ncp;
        v.coef64 = alloc<double>(cnt);
        v.coef32 = alloc<float>(cnt);
        fill(v.coef64, (long long)cnt);
        fill(v.coef32, (long long)cnt);
        with_p([&](auto PC) {
            constexpr int P = decltype(PC)::value;
            hipLaunchKernelGGL(k_kron_to_stencil<P>, dim3(grid_for(v.N * Sn)), dim3(kBlock), 0, stream,
                               (const double*)v.K64, (const double*)v.M64, v.n, v.ncp, v.coef64, v.coef32);
        });
        check_launch();
    }
}

void igamg_ctx::setup(const igamg_geometry& g, int degree, int levels) {
    auto t0 = std::chrono::steady_clock::now();
    geom = g.kind;
    p = degree;
    if (geom == IGAMG_UNIT_SQUARE) {
        kind = OP_KRON2D;
        dim = 2;
    } else if (geom == IGAMG_QUARTER_ANNULUS || geom == IGAMG_QUARTER_ANNULUS_EXACT) {
        kind = OP_STENCIL2D;
        dim = 2;
        if (g.r_in != 0.0 || g.r_out != 0.0) {
            if (!(std::isfinite(g.r_in) && std::isfinite(g.r_out) && g.r_in > 0.0 && g.r_out > g.r_in))
                throw Error(IGAMG_EINVAL, "annulus radii must satisfy 0 < r_in < r_out");
            r_in = g.r_in;
            r_out = g.r_out;
        }
    } else if (geom == IGAMG_UNIT_CUBE) {
        kind = OP_KRON3D;
        dim = 3;
    } else {
        throw Error(IGAMG_EINVAL, "unknown geometry kind");
    }
    if (p < 1 || p > 5 || (dim == 3 && p > 3)) throw Error(IGAMG_EINVAL, "unsupported degree");
    if (opt.nu1 < 0 || opt.nu2 < 0 || opt.nu1 + opt.nu2 == 0) throw Error(IGAMG_EINVAL, "bad nu1/nu2");
    if (opt.mu < 1 || opt.mu > kMaxMu) throw Error(IGAMG_EINVAL, "cycle index mu must be in 1..4");
    if (opt.smoother != IGAMG_SMOOTH_MCGS && opt.smoother != IGAMG_SMOOTH_JACOBI &&
        opt.smoother != IGAMG_SMOOTH_LEXGS)
        throw Error(IGAMG_EINVAL, "unknown smoother");
    if (opt.smoother == IGAMG_SMOOTH_LEXGS && g.kind == IGAMG_UNIT_CUBE)
        throw Error(IGAMG_EINVAL, "lexicographic Gauss-Seidel is 2D only");
    if (opt.precision != IGAMG_FP64 && opt.precision != IGAMG_FP32_IR)
        throw Error(IGAMG_EINVAL, "bad precision");
    if (opt.pde < IGAMG_PDE_POISSON || opt.pde > IGAMG_PDE_ADVECTION_DIFFUSION)
        throw Error(IGAMG_EINVAL, "unknown operator");
    if (opt.pde != IGAMG_PDE_POISSON && dim != 2)
        throw Error(IGAMG_EINVAL, "the full elliptic operators are 2D");
    if (opt.stream) {
        stream = (hipStream_t)opt.stream;
    } else {
        IGAMG_HIP(hipStreamCreateWithFlags(&stream, hipStreamDefault));  // orders against the legacy stream
        own_stream = true;
    }
    if (kind == OP_KRON2D && (opt.stored_stencil || opt.pde != IGAMG_PDE_POISSON)) kind = OP_STENCIL2D;
    setup_levels(g.n_el, levels);
    if (assembled()) {
        setup_annulus();
    } else {
        setup_kron();
        setup_coarse();
        if (kind == OP_STENCIL2D) setup_kron_stencils();
    }
    if (kind == OP_STENCIL2D) setup_records();
    for (int l = 0; l <= L; ++l) {
        Level& v = lv[l];
        v.x64 = alloc<double>(v.N);
        v.b64 = alloc<double>(v.N);
        v.r64 = alloc<double>(v.N);
        v.x32 = alloc_padded32(v.N);
        v.b32 = alloc<float>(v.N);
        v.r32 = alloc<float>(v.N);
        fill(v.x64, v.N);
        fill(v.b64, v.N);
        fill(v.b32, v.N);
    }
    raise_kron3_lds();
    default_shapes();
    choose_tail();
    b = alloc<double>(lv[L].N);
    fill(b, lv[L].N);
    npartial = std::max<long long>(residual_blocks(L), 1024);
    partial = alloc<double>(npartial);
    scal = alloc<double>(8);
    coeffs = alloc<ExtrapCoeffs>(1);
    IGAMG_HIP(hipHostMalloc((void**)&host_scal, 8 * sizeof(double), hipHostMallocDefault));
    setup_diag();
    IGAMG_HIP(hipHostMalloc((void**)&host_coeffs, sizeof(ExtrapCoeffs), hipHostMallocDefault));
    set_bnorm(0.0);
    setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// n_modes < 0: the built-in right-hand side of the context's Section 4.3 problem.
void igamg_ctx::set_rhs_field(const double* modes, int n_modes) {
    Level& f = lv[L];
    std::vector<double> md;
    if (n_modes >= 0) md.assign(modes, modes + (size_t)n_modes * (dim + 2));
    for (double v : md)
        if (!std::isfinite(v)) throw Error(IGAMG_ENONFINITE, "non-finite mode table");
    double* dmodes = md.empty() ? nullptr : upload(md);
    if (dim == 2) {
        int q = p + 1;
        ElementTables E = element_tables(f.n_el, p, q);
        double* V = upload(E.V);
        double* pts = upload(E.pts);
        double* wts = upload(E.wts);
        const int NQ = f.n_el * q;
        long long nqp = (long long)NQ * NQ;
        GeomQP G{};
        G.D11 = alloc<double>(nqp);
        G.D12 = alloc<double>(nqp);
        G.D22 = alloc<double>(nqp);
        G.wdet = alloc<double>(nqp);
        G.X = alloc<double>(nqp);
        G.Y = alloc<double>(nqp);
        double* fq = alloc<double>(nqp);
        GeomParams gp = geom_params();
        gp.pde = IGAMG_PDE_POISSON;  // only the geometry is needed
        hipLaunchKernelGGL(k_geometry_qp, dim3(grid_for(nqp)), dim3(kBlock), 0, stream, gp, NQ, pts, wts,
                           G);
        if (n_modes >= 0)
            hipLaunchKernelGGL(k_load_qp, dim3(grid_for(nqp)), dim3(kBlock), 0, stream, nqp, G, dmodes,
                               n_modes, fq);
        else
            hipLaunchKernelGGL(k_load_qp_builtin, dim3(grid_for(nqp)), dim3(kBlock), 0, stream, nqp, G,
                               opt.pde, fq);
        hipLaunchKernelGGL(k_assemble_load2d, dim3(grid_for(f.N)), dim3(kBlock), 0, stream, f.n_el, p,
                           q, V, fq, b);
        check_launch();
        sync();
        for (double* a : {G.D11, G.D12, G.D22, G.wdet, G.X, G.Y, fq, V, pts, wts}) release(a);
    } else {
        int q = p + 1;
        ElementTables E = element_tables(f.n_el, p, q);
        double* V = upload(E.V);
        double* pts = upload(E.pts);
        double* wts = upload(E.wts);
        hipLaunchKernelGGL(k_assemble_load3d, dim3(grid_for(f.N)), dim3(kBlock), 0, stream, f.n_el, p,
                           q, V, pts, wts, dmodes, n_modes, b);
        check_launch();
        sync();
        for (double* a : {V, pts, wts}) release(a);
    }
    if (dmodes) release(dmodes);
    set_bnorm(vector_norm(b, f.N));
}

// ---------------------------------------------------------------------------
// autotuning of the multi-block / single-workgroup split

// ---------------------------------------------------------------------------
// flexible GMRES with the (extrapolated) multigrid cycle as preconditioner

// z = M(v): one FP64 V-cycle from zero, or one RRE/MPE(q) restart cycle for
// A z = v from zero (the context's right-hand side is replaced by v for the
// cycle; the captured restart graph reads it from the same buffer).
void igamg_ctx::precond_apply(int precond, int q, const double* v, double* z) {
    const long long N = lv[L].N;
    if (precond == IGAMG_PRECOND_VCYCLE) {
        fill(z, N);
        vcycle<double>(v, z);
        return;
    }
    copy(v, b, N);
    ensure_iterates(q);
    fill(S[0], N);
    run_restart_cycle(precond == IGAMG_PRECOND_RRE ? IGAMG_RRE : IGAMG_MPE, q, false);
    copy(S[0], z, N);
}

// Right-preconditioned flexible GMRES(m) on the finest level: Arnoldi with
// classical Gram-Schmidt applied twice, Givens rotations on the host, the
// preconditioned directions Z kept for the update x += Z y.  Stops when
// ||b - A x|| <= tol ||b|| at a restart (the Arnoldi estimate ends a cycle early).
void igamg_ctx::fgmres(double tol, int max_iters, int m, int precond, int q, double* x, igamg_stats& st) {
    const long long N = lv[L].N;
    have_state = false;  // the preconditioner's restart cycles reuse the checkpoint buffer
    while ((int)kry_V.size() < m + 1) kry_V.push_back(alloc<double>(N));
    while ((int)kry_Z.size() < m) kry_Z.push_back(alloc<double>(N));
    const unsigned nbk = (unsigned)std::min<long long>(grid_for(N), 512);
    if (!kry_w) kry_w = alloc<double>(N);
    if (!kry_h) kry_h = alloc<double>(kMaxKrylov + 2);
    if (!kry_partial) kry_partial = alloc<double>((size_t)512 * (kMaxKrylov + 1));
    if (!bsave) bsave = alloc<double>(N);
    copy(b, bsave, N);
    const double nb = bnorm > 0.0 ? bnorm : 1.0;
    int iters = 0;
    bool converged = false;
    auto restore = [&]() { copy(bsave, b, N); sync(); };
    try {
        for (;;) {
            residual<double, double>(L, bsave, x, kry_w, 0, nullptr);
            const double beta = vector_norm(kry_w, N);
            st.residual_checks++;
            st.rel_residual = beta / nb;
            if (!std::isfinite(beta)) throw Error(IGAMG_ENONFINITE, "non-finite residual");
            if (beta <= tol * nb) {
                converged = true;
                break;
            }
            if (iters >= max_iters) break;
            hipLaunchKernelGGL(k_scaled_copy, dim3(grid_for(N)), dim3(kBlock), 0, stream, kry_w, kry_V[0],
                               1.0 / beta, N);
            check_launch();
            std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
            auto Hat = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
            g[0] = beta;
            int k = 0;
            for (int j = 0; j < m && iters < max_iters; ++j) {
                precond_apply(precond, q, kry_V[j], kry_Z[j]);
                st.vcycles += (precond == IGAMG_PRECOND_VCYCLE) ? 1 : q + 1;
                residual<double, double>(L, nullptr, kry_Z[j], kry_w, 1, nullptr);  // w = A z_j
                VecPtrs Vp{};
                for (int i = 0; i <= j; ++i) Vp.v[i] = kry_V[i];
                std::vector<double> h(j + 1, 0.0), hp(j + 1);
                for (int pass = 0; pass < 2; ++pass) {
                    hipLaunchKernelGGL(k_dots_partial, dim3(nbk), dim3(kBlock), 0, stream, (const double*)kry_w,
                                       Vp, j + 1, N, kry_partial);
                    hipLaunchKernelGGL(k_dots_finalize, dim3(1), dim3(64), 0, stream,
                                       (const double*)kry_partial, (int)nbk, j + 1, kry_h);
                    hipLaunchKernelGGL(k_axpy_multi, dim3(grid_for(N)), dim3(kBlock), 0, stream, kry_w, Vp,
                                       (const double*)kry_h, j + 1, -1.0, N);
                    check_launch();
                    IGAMG_HIP(hipMemcpyAsync(hp.data(), kry_h, (j + 1) * sizeof(double), hipMemcpyDeviceToHost,
                                             stream));
                    sync();
                    for (int i = 0; i <= j; ++i) h[i] += hp[i];
                }
                const double hn = vector_norm(kry_w, N);
                for (int i = 0; i <= j; ++i) Hat(i, j) = h[i];
                Hat(j + 1, j) = hn;
                if (hn > 0.0) {
                    hipLaunchKernelGGL(k_scaled_copy, dim3(grid_for(N)), dim3(kBlock), 0, stream, kry_w,
                                       kry_V[j + 1], 1.0 / hn, N);
                    check_launch();
                }
                for (int i = 0; i < j; ++i) {  // previous rotations on column j
                    const double a = Hat(i, j), c2 = Hat(i + 1, j);
                    Hat(i, j) = cs[i] * a + sn[i] * c2;
                    Hat(i + 1, j) = -sn[i] * a + cs[i] * c2;
                }
                const double r = std::hypot(Hat(j, j), Hat(j + 1, j));
                cs[j] = r > 0.0 ? Hat(j, j) / r : 1.0;
                sn[j] = r > 0.0 ? Hat(j + 1, j) / r : 0.0;
                Hat(j, j) = r;
                Hat(j + 1, j) = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                k = j + 1;
                ++iters;
                if (!std::isfinite(g[j + 1])) throw Error(IGAMG_ENONFINITE, "non-finite Arnoldi step");
                if (std::fabs(g[j + 1]) <= tol * nb || hn == 0.0) break;
            }
            std::vector<double> y(k, 0.0);
            for (int i = k - 1; i >= 0; --i) {
                double s = g[i];
                for (int l = i + 1; l < k; ++l) s -= Hat(i, l) * y[l];
                y[i] = s / Hat(i, i);
            }
            IGAMG_HIP(hipMemcpyAsync(kry_h, y.data(), k * sizeof(double), hipMemcpyHostToDevice, stream));
            VecPtrs Zp{};
            for (int i = 0; i < k; ++i) Zp.v[i] = kry_Z[i];
            hipLaunchKernelGGL(k_axpy_multi, dim3(grid_for(N)), dim3(kBlock), 0, stream, x, Zp,
                               (const double*)kry_h, k, 1.0, N);
            check_launch();
        }
    } catch (...) {
        restore();
        throw;
    }
    restore();
    st.restarts = iters;
    if (!converged) throw Error(IGAMG_ENOCONV, "tolerance not reached within max_iters");
}

// Autotuner: picks, by timing on the device, (1) per level the sweep launch
// shape (row-class launches or one launch per colour) in the current
// precision, (2) per level the learned inference kernel (the timing does not
// depend on the weights, so zero weights stand in), (3) the split between
// multi-block levels and the single-workgroup kernel (whole V-cycles with the
// choices of (1) and (2)); the result is cached for the process.
void igamg_ctx::autotune(int* best_items, double* best_ms, bool tune_learned) {
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    IGAMG_HIP(hipEventCreate(&ev.a));
    IGAMG_HIP(hipEventCreate(&ev.b));
    // ms of one replay of the launches `body` enqueues, captured as a graph
    // and replayed once to warm up, then once between two events
    auto timed = [&](auto&& body) -> double {
        hipGraph_t gr = nullptr;
        hipGraphExec_t ge = nullptr;
        IGAMG_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
            body();
        } catch (...) {
            hipGraph_t g2 = nullptr;
            (void)hipStreamEndCapture(stream, &g2);
            if (g2) (void)hipGraphDestroy(g2);
            throw;
        }
        IGAMG_HIP(hipStreamEndCapture(stream, &gr));
        float ms = 0.f;
        hipError_t err = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        if (err == hipSuccess) err = hipGraphLaunch(ge, stream);
        if (err == hipSuccess) err = hipEventRecord(ev.a, stream);
        if (err == hipSuccess) err = hipGraphLaunch(ge, stream);
        if (err == hipSuccess) err = hipEventRecord(ev.b, stream);
        if (err == hipSuccess) err = hipEventSynchronize(ev.b);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev.a, ev.b);
        if (ge) (void)hipGraphExecDestroy(ge);
        (void)hipGraphDestroy(gr);
        if (err != hipSuccess) throw Error(IGAMG_EHIP, std::string("autotune: ") + hipGetErrorString(err));
        return ms;
    };
    // (1) sweep launch shape per level
    auto sweep_shapes = [&](auto tag) {
        using T = decltype(tag);
        for (int l = 1; l <= L; ++l) {
            if (!row_sweeps_available(l)) continue;
            Level& v = lv[l];
            fill(v.x<T>(), v.N);
            hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(v.N)), dim3(kBlock), 0, stream, v.b<T>(), (T)1, v.N);
            check_launch();
            // stored stencils: one launch per colour or per row class (the
            // same iterates); sum-factorised operators: per row class, or (3D)
            // per plane class (the same iterates; one launch per colour sums
            // in another order and is not a candidate)
            const int lo = (kind == OP_STENCIL2D) ? 0 : 1, hi = plane3_available(l) ? 2 : 1;
            if (hi == lo) {
                row_pref[l] = lo;
                continue;
            }
            double t[3] = {1e300, 1e300, 1e300};
            for (int trial = 0; trial < 2; ++trial)
                for (int pref = lo; pref <= hi; ++pref) {
                    row_pref[l] = pref;
                    t[pref] = std::min(t[pref], timed([&] {
                        for (int k = 0; k < 4; ++k) mc_sweep<T>(l, v.b<T>(), v.x<T>());
                    }));
                }
            int best = hi;
            for (int pref = hi - 1; pref >= lo; --pref)
                if (t[pref] < t[best]) best = pref;
            row_pref[l] = best;
        }
    };
    if (opt.precision == IGAMG_FP64)
        sweep_shapes(double{});
    else
        sweep_shapes(float{});
    // (2) learned inference kernel per level
    if (dim == 2 && tune_learned) {
        const long long nmax = lv[L].N;
        float* zt = alloc<float>(nmax);
        float* yt = alloc<float>(nmax);
        fill(zt, nmax);
        Net tmp;
        tmp.wc = alloc<uint16_t>(kLWeights);
        tmp.w2f = alloc<uint16_t>(kLW2);
        tmp.w2b = alloc<uint16_t>(kLW2);
        tmp.mf32 = alloc<float>(kLMf32);
        tmp.mfbf = alloc<uint16_t>(kLMfBf);
        fill(tmp.wc, kLWeights);
        fill(tmp.w2f, kLW2);
        fill(tmp.w2b, kLW2);
        fill(tmp.mf32, kLMf32);
        fill(tmp.mfbf, kLMfBf);
        const int cand[] = {0, 12, 28, 29};
        for (int l = 1; l <= L; ++l) {
            const LImage im{zt, lv[l].n, lv[l].n, lv[l].n, 0, 0};
            double bt = 1e300;
            int bk = learned_kern[l];
            for (int k : cand) {
                // the better of two timed replays of 8 launches each
                double t = 1e300;
                for (int trial = 0; trial < 2; ++trial)
                    t = std::min(t, timed([&] {
                        for (int r = 0; r < 8; ++r)
                            learned_apply_k<float>(k, tmp, im, nullptr, (float*)nullptr, yt);
                    }));
                if (t < bt) {
                    bt = t;
                    bk = k;
                }
            }
            learned_kern[l] = bk;
        }
        for (void* q : {(void*)zt, (void*)yt, (void*)tmp.wc, (void*)tmp.w2f, (void*)tmp.w2b, (void*)tmp.mf32,
                        (void*)tmp.mfbf})
            release(q);
    }
    // (3) the multi-block / single-workgroup split
    const int cand[] = {0, 8, 16, 32, 64, 128, 256, 512};
    double* x = alloc<double>(lv[L].N);
    int save_items = opt.tail_items;
    int best = save_items;
    double bms = 1e300;
    int last_top = -1;
    for (int items : cand) {
        opt.tail_items = items;
        choose_tail();
        if (tail_top == last_top) continue;  // same split as a smaller threshold
        last_top = tail_top;
        fill(x, lv[L].N);
        G(x);  // warm-up
        IGAMG_HIP(hipEventRecord(ev.a, stream));
        for (int k = 0; k < 3; ++k) G(x);
        IGAMG_HIP(hipEventRecord(ev.b, stream));
        IGAMG_HIP(hipEventSynchronize(ev.b));
        float ms = 0.f;
        IGAMG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        if (ms / 3.0 < bms) {
            bms = ms / 3.0;
            best = items;
        }
    }
    release(x);
    opt.tail_items = best;
    choose_tail();
    graph_method = -1;
    tuned_ms = bms;
    {
        TuneChoice c;
        c.tail_items = best;
        c.row = row_pref;
        c.learned = learned_kern;
        c.vcycle_ms = bms;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[tune_key()] = c;
    }
    if (best_items) *best_items = best;
    if (best_ms) *best_ms = bms;
}

// ---------------------------------------------------------------------------
// learned smoother: diagonals, level solves, training

void igamg_ctx::setup_diag() {
    diag64.assign(L + 1, nullptr);
    diag32.assign(L + 1, nullptr);
    for (int l = 0; l <= L; ++l) {
        Level& v = lv[l];
        diag64[l] = alloc<double>(v.N);
        diag32[l] = alloc<float>(v.N);
        if (kind == OP_STENCIL2D) {
            with_p([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                hipLaunchKernelGGL(k_diag_stencil<P>, dim3(grid_for(v.N)), dim3(kBlock), 0, stream,
                                   v.coef64, v.n, v.ncp, diag64[l], diag32[l]);
            });
            check_launch();
        } else {
            std::vector<double> d(v.N);
            std::vector<float> d32(v.N);
            int n = v.n;
            for (long long I = 0; I < v.N; ++I) {
                int i = (int)(I % n), j = (int)((I / n) % n), k = (int)(I / ((long long)n * n));
                double val = (dim == 2)
                                 ? v.Kh.at(i, 0) * v.Mh.at(j, 0) + v.Mh.at(i, 0) * v.Kh.at(j, 0)
                                 : v.Kh.at(i, 0) * v.Mh.at(j, 0) * v.Mh.at(k, 0) +
                                       v.Mh.at(i, 0) * v.Kh.at(j, 0) * v.Mh.at(k, 0) +
                                       v.Mh.at(i, 0) * v.Mh.at(j, 0) * v.Kh.at(k, 0);
                d[I] = val;
                d32[I] = (float)val;
            }
            IGAMG_HIP(hipMemcpyAsync(diag64[l], d.data(), d.size() * 8, hipMemcpyHostToDevice, stream));
            IGAMG_HIP(hipMemcpyAsync(diag32[l], d32.data(), d32.size() * 4, hipMemcpyHostToDevice, stream));
            sync();
        }
    }
    lz = alloc<float>(lv[L].N);
    nets.assign(L + 1, Net{});
}

void igamg_ctx::ensure_net(int l) {
    Net& t = nets[l];
    if (t.wc) return;
    t.wc = alloc<uint16_t>(kLWeights);
    t.w2f = alloc<uint16_t>(kLW2);
    t.w2b = alloc<uint16_t>(kLW2);
    t.mf32 = alloc<float>(kLMf32);
    t.mfbf = alloc<uint16_t>(kLMfBf);
    fill(t.mf32, kLMf32);  // record entries of no weight stay zero
    fill(t.mfbf, kLMfBf);
    t.master = alloc<float>(kLWeights);
    t.m = alloc<float>(kLWeights);
    t.v = alloc<float>(kLWeights);
}

// ||f - A_l x|| / fnorm on level l (host value).
double igamg_ctx::level_resnorm(int l, const double* f, const double* x, double fnorm) {
    residual<double, double>(l, f, x, lv[l].r64, 0, partial);
    long long nb = residual_blocks(l);
    hipLaunchKernelGGL(k_finalize_norm, dim3(1), dim3(kBlock), 0, stream, partial, (int)nb,
                       fnorm > 0 ? fnorm : 1.0, (const double*)nullptr, scal);
    check_launch();
    return read_scal();
}

// Plain FP64 V-cycles from level l until ||f - A u|| <= tol ||f||; u holds the
// initial guess.  Returns the number of cycles (level 0: direct solve).
int igamg_ctx::level_solve(int l, const double* f, double* u, double tol, int maxit) {
    if (l == 0) {
        coarse<double>(f, u);
        return 0;
    }
    double fn = vector_norm(f, lv[l].N);
    if (fn == 0.0) {
        fill(u, lv[l].N);
        return 0;
    }
    for (int k = 1; k <= maxit; ++k) {
        vcycle_from<double>(l, f, u);
        if (level_resnorm(l, f, u, fn) <= tol) return k;
    }
    return maxit;
}

// Geometric-mean residual contraction per V-cycle over the second half of
// `vcycles` plain FP64 V-cycles from zero on the current right-hand side.
double igamg_ctx::measure_rho(int vcycles, bool learned) {
    bool save = learned_on;
    learned_on = learned;
    double* x = alloc<double>(lv[L].N);
    fill(x, lv[L].N);
    int h = vcycles / 2;
    double r_h = 0.0, r_e = 0.0;
    for (int k = 1; k <= vcycles; ++k) {
        vcycle<double>(b, x);
        if (k == h || k == vcycles) {
            resnorm_async(x);
            double r = read_scal();
            if (k == h) r_h = r; else r_e = r;
        }
    }
    release(x);
    learned_on = save;
    if (!(r_h > 0.0) || !(r_e > 0.0)) return 0.0;
    return std::pow(r_e / r_h, 1.0 / (vcycles - h));
}

// The same measure for the cycle started on level l (levels 0..l) with
// right-hand side f of level l.
double igamg_ctx::measure_rho_level(int l, const double* f, int vcycles, bool learned) {
    bool save = learned_on;
    learned_on = learned;
    double* u = alloc<double>(lv[l].N);
    fill(u, lv[l].N);
    int h = vcycles / 2;
    double r_h = 0.0, r_e = 0.0;
    for (int k = 1; k <= vcycles; ++k) {
        vcycle_from<double>(l, f, u);
        if (k == h) r_h = level_resnorm(l, f, u, 1.0);
        if (k == vcycles) r_e = level_resnorm(l, f, u, 1.0);
    }
    release(u);
    learned_on = save;
    if (!(r_h > 0.0) || !(r_e > 0.0)) return 0.0;
    return std::pow(r_e / r_h, 1.0 / (vcycles - h));
}

void igamg_ctx::train(const igamg_train_options& o, igamg_train_report& rep) {
    auto t0 = std::chrono::steady_clock::now();
    if (dim != 2) throw Error(IGAMG_EINVAL, "the learned smoother is 2D only");
    if (o.n_rhs < 1 || !o.modes || o.n_modes < 1 || o.vcycles_per_rhs < 1 || o.epochs < 1 ||
        o.batch < 1 || !(o.lr > 0) || o.val_vcycles < 4 || !(o.solve_tol > 0))
        throw Error(IGAMG_EINVAL, "bad training options");
    const long long NL = lv[L].N;
    // keep the user's right-hand side and settings
    double* bsave = alloc<double>(NL);
    copy(b, bsave, NL);
    double bnorm_save = bnorm;
    int tail_save = tail_top, prec_save = opt.precision;
    bool learned_save = learned_on;
    tail_top = 0;
    learned_on = false;
    opt.precision = IGAMG_FP64;

    // ---- samples: per level lists of (z, t) FP32 full-level vectors
    std::vector<std::vector<std::pair<float*, float*>>> samples(L + 1);
    double* ustar = alloc<double>(NL);
    double* xw = alloc<double>(NL);
    double* tmp1 = alloc<double>(NL);
    double* tmp2 = alloc<double>(NL);
    double* tmp3 = alloc<double>(NL);
    double* tmp4 = alloc<double>(NL);
    for (int k = 0; k < o.n_rhs; ++k) {
        set_rhs_field(o.modes + (size_t)k * o.n_modes * (dim + 2), o.n_modes);
        fill(ustar, NL);
        level_solve(L, b, ustar, o.solve_tol, 2000);
        fill(xw, NL);
        for (int v = 0; v < o.vcycles_per_rhs; ++v) {
            // snapshot (b_l, x_l) at the entry of every level >= 1
            std::vector<std::tuple<int, double*, double*>> snaps;
            vcycle_from<double>(L, b, xw, [&](int l, const double* bl, double* xl) {
                double* sb = alloc<double>(lv[l].N);
                double* sx = alloc<double>(lv[l].N);
                copy(bl, sb, lv[l].N);
                copy((const double*)xl, sx, lv[l].N);
                snaps.emplace_back(l, sb, sx);
            });
            for (auto& sn : snaps) {
                int l = std::get<0>(sn);
                double* sb = std::get<1>(sn);
                double* sx = std::get<2>(sn);
                Level& lvv = lv[l];
                long long N = lvv.N;
                // r = b_l - A_l x_l  (tmp1), u_l (tmp2), e = u_l - x_l (tmp3)
                residual<double, double>(l, sb, sx, tmp1, 0, nullptr);
                if (l == L) {
                    copy(ustar, tmp2, N);
                } else {
                    fill(tmp2, N);
                    level_solve(l, sb, tmp2, o.solve_tol, 2000);
                }
                hipLaunchKernelGGL(k_sub, dim3(grid_for(N)), dim3(kBlock), 0, stream, tmp2, sx, tmp3, N);
                // e_c = A_{l-1}^{-1} R r, then t = e - P e_c
                Level& cl = lv[l - 1];
                double* rc = alloc<double>(cl.N);
                double* ec = alloc<double>(cl.N);
                restrict_<double>(l, tmp1, rc);
                fill(ec, cl.N);
                level_solve(l - 1, rc, ec, o.solve_tol, 2000);
                fill(tmp4, N);
                prolong_<double>(l, ec, tmp4);
                hipLaunchKernelGGL(k_sub, dim3(grid_for(N)), dim3(kBlock), 0, stream, tmp3, tmp4, tmp2, N);
                // sigma = RMS(D^{-1} r); pack
                unsigned nb = grid_for(N);
                hipLaunchKernelGGL(k_learned_sumsq_scaled, dim3(nb), dim3(kBlock), 0, stream, tmp1,
                                   diag64[l], N, partial);
                hipLaunchKernelGGL(k_learned_sigma, dim3(1), dim3(kLSigmaThreads), 0, stream, partial, (int)nb, N,
                                   scal + 3);
                float* zz = alloc<float>(N);
                float* tt = alloc<float>(N);
                hipLaunchKernelGGL(k_learned_pack, dim3(nb), dim3(kBlock), 0, stream, tmp1, diag64[l],
                                   tmp2, N, (const double*)(scal + 3), zz, tt);
                check_launch();
                samples[l].push_back({zz, tt});
                release(rc);
                release(ec);
                release(sb);
                release(sx);
            }
            sync();
        }
    }
    for (double* a : {ustar, xw, tmp1, tmp2, tmp3, tmp4}) release(a);

    // ---- patches and training per level
    std::vector<double> lfirst(L + 1, 0.0), llast(L + 1, 0.0);
    unsigned long long rng = o.seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto rnd = [&]() {
        rng = rng * 6364136223846793005ULL + 1442695040888963407ULL;
        return (uint32_t)(rng >> 33);
    };
    auto gauss = [&]() {
        double u1 = (rnd() + 1.0) / 4294967297.0, u2 = (rnd() + 1.0) / 4294967297.0;
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    int total_patches = 0, trained = 0;
    for (int l = 1; l <= L; ++l) {
        if (samples[l].empty()) continue;
        if (l <= tail_save) {  // run by the single-workgroup kernel: keeps Gauss-Seidel
            for (auto& sm : samples[l]) {
                release(sm.first);
                release(sm.second);
            }
            continue;
        }
        Level& v = lv[l];
        int n = v.n, ls = std::min(64, n), W = ls + 6;
        int tpr = (n + ls - 1) / ls;
        std::vector<float*> pz, pt;
        for (auto& sm : samples[l]) {
            for (int a = 0; a < tpr; ++a)
                for (int c = 0; c < tpr; ++c) {
                    float* z = alloc<float>((size_t)W * W);
                    float* t = alloc<float>((size_t)ls * ls);
                    hipLaunchKernelGGL(k_learned_cut, dim3((W * W + 255) / 256), dim3(256), 0, stream,
                                       sm.first, sm.second, n, a * ls, c * ls, ls, z, t);
                    pz.push_back(z);
                    pt.push_back(t);
                }
            release(sm.first);
            release(sm.second);
        }
        check_launch();
        int np = (int)pz.size();
        total_patches += np;
        // initial weights: scaled normal (same scale rule as the oracle's init)
        ensure_net(l);
        Net& net = nets[l];
        std::vector<float> w0(kLWeights);
        for (int k = 0; k < kLW1; ++k) w0[k] = (float)(gauss() * std::sqrt(2.0 / 9.0));
        for (int k = 0; k < kLW2; ++k) w0[kLW1 + k] = (float)(gauss() * std::sqrt(2.0 / 144.0));
        for (int k = 0; k < kLW3; ++k) w0[kLW1 + kLW2 + k] = (float)(0.1 * gauss() * std::sqrt(2.0 / 144.0));
        IGAMG_HIP(hipMemcpyAsync(net.master, w0.data(), kLWeights * 4, hipMemcpyHostToDevice, stream));
        fill(net.m, kLWeights);
        fill(net.v, kLWeights);
        // BF16 copies through one zero-gradient Adam call with lr = 0
        float* g = alloc<float>(kLWeights);
        fill(g, kLWeights);
        hipLaunchKernelGGL(k_learned_adam, dim3((kLWeights + 255) / 256), dim3(256), 0, stream, net.master,
                           net.m, net.v, (const float*)g, 0.f, 0.9f, 0.999f, 1e-8f, 1.f, 1.f, net.wc, net.w2f,
                           net.w2b, net.mf32, net.mfbf);
        net.have = true;
        net.on = true;
        int tiles = ((ls + kLTile - 1) / kLTile) * ((ls + kLTile - 1) / kLTile);
        int B = std::min(o.batch, np);
        float* gpart = alloc<float>((size_t)B * tiles * kLWeights);
        double* lpart = alloc<double>((size_t)B * tiles);
        double* lsum = alloc<double>(1);
        LItem* ditems = alloc<LItem>(B);
        std::vector<LItem> hitems(B);
        std::vector<int> order(np);
        for (int k = 0; k < np; ++k) order[k] = k;
        int step = 0;
        for (int ep = 0; ep < o.epochs; ++ep) {
            for (int k = np - 1; k > 0; --k) std::swap(order[k], order[rnd() % (k + 1)]);
            double eloss = 0.0;
            int ebatches = 0;
            for (int s0 = 0; s0 + B <= np; s0 += B) {
                for (int k = 0; k < B; ++k) {
                    int pidx = order[s0 + k];
                    int a = pidx % (tpr * tpr);
                    int j0 = (a / tpr) * ls, i0 = (a % tpr) * ls;
                    hitems[k].im = LImage{pz[pidx], W, W, n, i0 - 3, j0 - 3};
                    hitems[k].t = pt[pidx];
                    hitems[k].l0 = 3;
                    hitems[k].lsize = ls;
                }
                IGAMG_HIP(hipMemcpyAsync(ditems, hitems.data(), B * sizeof(LItem), hipMemcpyHostToDevice,
                                         stream));
                // loss pixels of the batch (inside the domain)
                long long cnt = 0;
                for (int k = 0; k < B; ++k) {
                    int j0 = hitems[k].im.off_j + 3, i0 = hitems[k].im.off_i + 3;
                    cnt += (long long)std::min(ls, n - j0) * std::min(ls, n - i0);
                }
                LearnedW Wd{net.wc, net.w2f, net.w2b};
                hipLaunchKernelGGL(k_learned_train, dim3(B * tiles), dim3(kLThreads), 0, stream,
                                   (const LItem*)ditems, tiles, Wd, (float)(1.0 / cnt), gpart, lpart);
                hipLaunchKernelGGL(k_learned_reduce, dim3((kLWeights + 255) / 256), dim3(256), 0, stream,
                                   (const float*)gpart, B * tiles, (const double*)lpart, g, lsum);
                ++step;
                float bc1 = 1.f - std::pow(0.9f, (float)step), bc2 = 1.f - std::pow(0.999f, (float)step);
                hipLaunchKernelGGL(k_learned_adam, dim3((kLWeights + 255) / 256), dim3(256), 0, stream,
                                   net.master, net.m, net.v, (const float*)g, (float)o.lr, 0.9f, 0.999f,
                                   1e-8f, bc1, bc2, net.wc, net.w2f, net.w2b, net.mf32, net.mfbf);
                check_launch();
                if (ep == 0 || ep == o.epochs - 1) {
                    IGAMG_HIP(hipMemcpyAsync(host_scal + 4, lsum, 8, hipMemcpyDeviceToHost, stream));
                    sync();
                    eloss += host_scal[4] / cnt;
                    ++ebatches;
                }
            }
            if (ep == 0) lfirst[l] = ebatches ? eloss / ebatches : 0.0;
            if (ep == o.epochs - 1) llast[l] = ebatches ? eloss / ebatches : 0.0;
        }
        sync();
        for (float* a : pz) release(a);
        for (float* a : pt) release(a);
        release(gpart);
        release(lpart);
        release(lsum);
        release(ditems);
        release(g);
        ++trained;
    }
    // ---- validation: contraction with and without the networks
    tail_top = tail_save;
    if (o.val_modes)
        set_rhs_field(o.val_modes, o.val_n_modes);
    else
        set_rhs_field(o.modes, o.n_modes);
    double rp = measure_rho(o.val_vcycles, false);
    double rl = 0.0;
    {
        // per level: the cycle started on level l, right-hand side R^(L-l) b
        std::vector<double*> f(L + 1, nullptr);
        f[L] = b;
        for (int l = L; l >= 2; --l) {
            f[l - 1] = alloc<double>(lv[l - 1].N);
            restrict_<double>(l, f[l], f[l - 1]);
        }
        // per_level_accept, bottom-up: level l keeps its network only if the
        // cycle started on level l contracts better with it than without (the
        // levels below as already decided)
        for (int l = 0; l < 16; ++l) rep.accepted_level[l] = 0;
        for (int l = 1; l <= L; ++l) {
            if (l <= tail_top || l >= (int)nets.size() || !nets[l].have) continue;
            if (o.per_level_accept) {
                nets[l].on = false;
                const double off = measure_rho_level(l, f[l], o.val_vcycles, true);
                nets[l].on = true;
                const double on = measure_rho_level(l, f[l], o.val_vcycles, true);
                if (!(on > 0.0 && on < off)) nets[l].on = false;
            }
            if (l < 16) rep.accepted_level[l] = nets[l].on ? 1 : 0;
        }
        rl = measure_rho(o.val_vcycles, true);
        for (int l = 0; l < 16; ++l) rep.rho_plain_level[l] = rep.rho_learned_level[l] = 0.0;
        for (int l = 1; l <= L && l < 16; ++l) {
            rep.rho_plain_level[l] = (l == L) ? rp : measure_rho_level(l, f[l], o.val_vcycles, false);
            rep.rho_learned_level[l] = (l == L) ? rl : measure_rho_level(l, f[l], o.val_vcycles, true);
        }
        for (int l = 1; l < L; ++l) release(f[l]);
    }
    rep.levels_trained = trained;
    rep.patches = total_patches;
    for (int l = 0; l < 16; ++l) {
        rep.loss_first[l] = (l <= L) ? lfirst[l] : 0.0;
        rep.loss_last[l] = (l <= L) ? llast[l] : 0.0;
    }
    rep.rho_plain = rp;
    rep.rho_learned = rl;
    rep.accepted = (rl > 0.0 && rl < rp) ? 1 : 0;
    rho_plain_ref = rp;
    // restore the user's state; enable the networks only if they contract better
    copy(bsave, b, NL);
    release(bsave);
    set_bnorm(bnorm_save);
    opt.precision = prec_save;
    learned_on = rep.accepted ? true : learned_save;
    graph_method = -1;
    sync();
    rep.train_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------------------
// batches of independent 2D problems

#define BLAUNCH(...) do { if (!preparing) hipLaunchKernelGGL(__VA_ARGS__); } while (0)

struct igamg_batch {
    std::vector<igamg_ctx*> inst;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<hipStream_t> side;  // one per degree group (graph branches)
    std::vector<hipEvent_t> ev;
    // argument tables of the captured plan: packed on the host by the prepare
    // pass, uploaded in one copy into a device buffer kept (and grown) across plans
    std::vector<unsigned char> plan_host;
    std::vector<size_t> plan_offs;
    unsigned char* plan_dev = nullptr;
    size_t plan_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int> plan_active;
    int plan_q = -1;
    double* rel_dev = nullptr;
    double* rel_host = nullptr;
    const double** scal_ptrs = nullptr;

    ~igamg_batch() {
        clear_plan();
        destroy_retired();
        if (plan_dev) (void)hipFree(plan_dev);
        for (auto* c : inst) delete c;
        for (auto e : ev) (void)hipEventDestroy(e);
        for (auto st : side) (void)hipStreamDestroy(st);
        if (rel_host) (void)hipHostFree(rel_host);
        if (rel_dev) (void)hipFree(rel_dev);
        if (scal_ptrs) (void)hipFree((void*)scal_ptrs);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    // Graphs of earlier plans, idle (every round ends with a stream
    // synchronisation), destroyed after the next plan's launch so that their
    // host-side teardown overlaps the GPU's work.
    std::vector<hipGraphExec_t> retired_exec;
    std::vector<hipGraph_t> retired_graph;
    void destroy_retired() {
        for (auto e : retired_exec) (void)hipGraphExecDestroy(e);
        for (auto g : retired_graph) (void)hipGraphDestroy(g);
        retired_exec.clear();
        retired_graph.clear();
    }
    void clear_plan() {
        if (gexec) retired_exec.push_back(gexec);
        if (graph) retired_graph.push_back(graph);
        gexec = nullptr;
        graph = nullptr;
        plan_host.clear();
        plan_offs.clear();
        plan_active.clear();
        plan_q = -1;
    }
    // Tables are built in a prepare pass (packed on the host, nothing launched),
    // uploaded once (upload_plan), and handed out in the same order by the
    // capture pass.
    bool preparing = false;
    size_t cursor = 0;
    template <typename E>
    const E* up(const std::vector<E>& v) {
        if (!preparing) return reinterpret_cast<const E*>(plan_dev + plan_offs.at(cursor++));
        const size_t off = (plan_host.size() + 15) & ~(size_t)15;
        const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(E);
        plan_host.resize(off + bytes, 0);
        if (!v.empty()) std::memcpy(plan_host.data() + off, v.data(), v.size() * sizeof(E));
        plan_offs.push_back(off);
        return nullptr;  // (the prepare pass launches nothing)
    }
    // One copy of the packed tables; the previous plan's graph has finished
    // (every round ends with a stream synchronisation).
    void upload_plan() {
        const size_t need = std::max<size_t>(plan_host.size(), 16);
        if (need > plan_cap) {
            if (plan_dev) IGAMG_HIP(hipFree(plan_dev));
            plan_dev = nullptr;
            plan_cap = 0;
            IGAMG_HIP(hipMalloc((void**)&plan_dev, need + need / 2));
            plan_cap = need + need / 2;
        }
        IGAMG_HIP(hipMemcpy(plan_dev, plan_host.data(), plan_host.size(), hipMemcpyHostToDevice));
    }
    // prefix offsets of per-entry block counts
    const int* offsets(const std::vector<int>& counts, int& total) {
        std::vector<int> o(counts.size() + 1, 0);
        for (size_t i = 0; i < counts.size(); ++i) o[i + 1] = o[i] + counts[i];
        total = o.back();
        return up(o);
    }

    // One launch per step of the FP32-in-FP64 map G for all `mem` problems of
    // degree P on stream st: G(W) = W + V32(round32(b - A64 W)), W = lv[L].x64.
    template <int P>
    void group_G(const std::vector<int>& mem, hipStream_t st) {
        using Op64 = Stencil2D<P, double>;
        using Op32 = Stencil2D<P, float>;
        constexpr int NC = Op32::NC;
        const int ne = (int)mem.size();
        int D = 0;
        for (int i : mem) D = std::max(D, inst[i]->L);
        // fine-level FP64 residual into b32, zero x32
        {
            std::vector<BRes<Op64, float>> E;
            std::vector<int> cnt;
            std::vector<BVec> Z;
            std::vector<int> zc;
            for (int i : mem) {
                igamg_ctx* c = inst[i];
                Level& f = c->lv[c->L];
                E.push_back({Op64{f.coef64, f.n, f.ncp}, c->b, f.x64, f.b32, f.N});
                cnt.push_back(NC * (f.ncp / 64));
                Z.push_back({nullptr, nullptr, f.x32, f.N});
                zc.push_back((int)grid_for(f.N));
            }
            int tot, ztot;
            const int* o = offsets(cnt, tot);
            const int* zo = offsets(zc, ztot);
            auto tb_E_1 = up(E);
            BLAUNCH((k_b_res<Op64, float>), dim3(tot), dim3(64 * Op64::NW), 0, st, tb_E_1, o, ne);
            auto tb_Z_2 = up(Z);
            BLAUNCH(k_b_vec, dim3(ztot), dim3(kBlock), 0, st, tb_Z_2, zo, ne, 0);
        }
        // per depth: smoothing tables (shared by descent and ascent)
        auto gs_tables = [&](int d, std::vector<int>& sel) {
            std::vector<BGs<Op32>> E;
            std::vector<int> offs((size_t)NC * 0);
            sel.clear();
            for (int k = 0; k < ne; ++k) {
                igamg_ctx* c = inst[mem[k]];
                int l = c->L - d;
                if (l <= c->tail_top) continue;
                sel.push_back(k);
                Level& v = c->lv[l];
                E.push_back({Op32{v.coef32, v.n, v.ncp}, v.b32, v.x32});
            }
            return E;
        };
        auto launch_sweeps = [&](int d, int nsweeps) {
            std::vector<int> sel;
            auto E = gs_tables(d, sel);
            if (E.empty() || nsweeps == 0) return;
            int nsel = (int)sel.size();
            std::vector<int> offs((size_t)NC * (nsel + 1), 0);
            std::vector<int> tot(NC, 0);
            for (int c = 0; c < NC; ++c) {
                for (int k = 0; k < nsel; ++k) {
                    igamg_ctx* cx = inst[mem[sel[k]]];
                    int cs = colour_size_host(cx->lv[cx->L - d].n, P, 2, c);
                    offs[(size_t)c * (nsel + 1) + k + 1] = offs[(size_t)c * (nsel + 1) + k] + (cs + 63) / 64;
                }
                tot[c] = offs[(size_t)c * (nsel + 1) + nsel];
            }
            const BGs<Op32>* dE = up(E);
            if constexpr (row_kernel_ok<Op32>()) {
                // one launch per row class: workgroup per row, sized for the
                // group's widest row (the same iterates as per-colour launches)
                bool rows = true;
                int th = 64;
                long long coef = 0;
                for (int k = 0; k < nsel; ++k) {
                    igamg_ctx* cx = inst[mem[sel[k]]];
                    const int l = cx->L - d;
                    rows = rows && cx->row_sweeps_available(l);
                    th = std::max(th, row_threads(P, cx->lv[l].n));
                    coef = std::max(coef, cx->coef_bytes(l, sizeof(float)));
                }
                if (rows) {
                    std::vector<int> ro((size_t)(P + 1) * (nsel + 1), 0);
                    std::vector<int> rt(P + 1, 0);
                    for (int r = 0; r <= P; ++r) {
                        for (int k = 0; k < nsel; ++k) {
                            igamg_ctx* cx = inst[mem[sel[k]]];
                            const int nj = (cx->lv[cx->L - d].n - r + P) / (P + 1);
                            ro[(size_t)r * (nsel + 1) + k + 1] = ro[(size_t)r * (nsel + 1) + k] + std::max(nj, 0);
                        }
                        rt[r] = ro[(size_t)r * (nsel + 1) + nsel];
                    }
                    const int* dR = up(ro);
                    const bool stream_coef = coef > igamg_ctx::kCachedCoefBytes;
                    for (int s2 = 0; s2 < nsweeps; ++s2)
                        for (int r = 0; r <= P; ++r) {
                            if (rt[r] <= 0) continue;
                            if (stream_coef)
                                BLAUNCH((k_b_rowclass<Op32, true>), dim3(rt[r]), dim3(th), 0, st, dE, dR, nsel, r);
                            else
                                BLAUNCH((k_b_rowclass<Op32, false>), dim3(rt[r]), dim3(th), 0, st, dE, dR, nsel,
                                        r);
                        }
                    return;
                }
            }
            const int* dO = up(offs);
            for (int s2 = 0; s2 < nsweeps; ++s2)
                for (int c = 0; c < NC; ++c)
                    if (tot[c] > 0)
                        BLAUNCH((k_b_gs<Op32>), dim3(tot[c]), dim3(64 * Op32::NW), 0, st, dE, dO,
                                           nsel, c);
        };
        for (int d = 0; d < D; ++d) {
            launch_sweeps(d, inst[mem[0]]->opt.nu1);
            std::vector<BRes<Op32, float>> R;
            std::vector<int> rc;
            std::vector<BTr<float>> T;
            std::vector<int> tc;
            for (int i : mem) {
                igamg_ctx* c = inst[i];
                int l = c->L - d;
                if (l <= c->tail_top) continue;
                Level& v = c->lv[l];
                Level& w = c->lv[l - 1];
                R.push_back({Op32{v.coef32, v.n, v.ncp}, v.b32, v.x32, v.r32, v.N});
                rc.push_back(NC * (v.ncp / 64));
                T.push_back({v.r32, w.b32, w.x32, v.n, w.n, v.r_start, v.r_w32, v.RW});
                tc.push_back((int)grid_for(w.N));
            }
            if (R.empty()) continue;
            int rt, tt;
            const int* ro = offsets(rc, rt);
            const int* to = offsets(tc, tt);
            auto tR = up(R);
            auto tT = up(T);
            BLAUNCH((k_b_res<Op32, float>), dim3(rt), dim3(64 * Op32::NW), 0, st, tR, ro, (int)R.size());
            BLAUNCH((k_b_restrict<Op32::kP, float>), dim3(tt), dim3(kBlock), 0, st, tT, to, (int)T.size());
        }
        {
            // every problem's small levels (and its coarsest solve): one workgroup each
            std::vector<TailArgs<Op32>> TA;
            for (int i : mem) {
                igamg_ctx* c = inst[i];
                int t = c->tail_top;
                TA.push_back(c->tail_args<Op32>(c->lv[t].b32, c->lv[t].x32));
            }
            auto tTA = up(TA);
            BLAUNCH((k_b_tail<Op32>), dim3(ne), dim3(tail_threads<Op32>()), 0, st, tTA);
        }
        for (int d = D - 1; d >= 0; --d) {
            std::vector<BTr<float>> T;
            std::vector<int> tc;
            for (int i : mem) {
                igamg_ctx* c = inst[i];
                int l = c->L - d;
                if (l <= c->tail_top) continue;
                Level& v = c->lv[l];
                Level& w = c->lv[l - 1];
                T.push_back({w.x32, v.x32, nullptr, v.n, w.n, v.p_start, v.p_w32, v.PW});
                tc.push_back((int)grid_for(v.N));
            }
            if (T.empty()) continue;
            int tt;
            const int* to = offsets(tc, tt);
            auto tb_T_6 = up(T);
            BLAUNCH((k_b_prolong<Op32::kP, float>), dim3(tt), dim3(kBlock), 0, st, tb_T_6, to, (int)T.size());
            launch_sweeps(d, inst[mem[0]]->opt.nu2);
        }
        // W += x32
        {
            std::vector<BVec> A;
            std::vector<int> ac;
            for (int i : mem) {
                igamg_ctx* c = inst[i];
                Level& f = c->lv[c->L];
                A.push_back({nullptr, f.x64, f.x32, f.N});
                ac.push_back((int)grid_for(f.N));
            }
            int at;
            const int* ao = offsets(ac, at);
            auto tb_A_7 = up(A);
            BLAUNCH(k_b_vec, dim3(at), dim3(kBlock), 0, st, tb_A_7, ao, ne, 2);
        }
    }

    // copies between each active problem's iterate buffers: mode 1, b64 = a64
    void copies(const std::vector<int>& act, int from, int to_) {
        std::vector<BVec> E;
        std::vector<int> c;
        for (int i : act) {
            igamg_ctx* x = inst[i];
            Level& f = x->lv[x->L];
            double* src = from < 0 ? f.x64 : x->S[from];
            double* dst = to_ < 0 ? f.x64 : x->S[to_];
            E.push_back({src, dst, nullptr, f.N});
            c.push_back((int)grid_for(f.N));
        }
        int tot;
        const int* o = offsets(c, tot);
        auto tb_E_8 = up(E);
        BLAUNCH(k_b_vec, dim3(tot), dim3(kBlock), 0, stream, tb_E_8, o, (int)act.size(), 1);
    }

    // Enqueue one restart cycle of every active problem.
    void restart_round(const std::vector<int>& act, int q) {
        std::vector<std::vector<int>> byp(6);
        for (int i : act) byp[inst[i]->p].push_back(i);
        copies(act, 0, -1);
        for (int j = 0; j <= q; ++j) {
            // fork: one branch per degree group
            int g = 0;
            if (!preparing) IGAMG_HIP(hipEventRecord(ev[0], stream));
            for (int pp = 1; pp <= 5; ++pp) {
                if (byp[pp].empty()) continue;
                hipStream_t st = side[g];
                if (!preparing) IGAMG_HIP(hipStreamWaitEvent(st, ev[0], 0));
                switch (pp) {
                    case 1: group_G<1>(byp[pp], st); break;
                    case 2: group_G<2>(byp[pp], st); break;
                    case 3: group_G<3>(byp[pp], st); break;
                    case 4: group_G<4>(byp[pp], st); break;
                    case 5: group_G<5>(byp[pp], st); break;
                }
                if (!preparing) IGAMG_HIP(hipEventRecord(ev[1 + g], st));
                ++g;
            }
            for (int k = 0; k < g && !preparing; ++k) IGAMG_HIP(hipStreamWaitEvent(stream, ev[1 + k], 0));
            copies(act, -1, j + 1);
        }
        for (int i : act) {
            if (preparing) break;
            igamg_ctx* c = inst[i];
            IterPtrs it = c->iter_ptrs(q);
            c->extrap_coeffs_async(it, q, IGAMG_RRE);
            long long N = c->lv[c->L].N;
            BLAUNCH(k_extrap_combine, dim3(grid_for(N)), dim3(kBlock), 0, stream, it, q, N,
                               (const ExtrapCoeffs*)c->coeffs, c->S[0], (double*)nullptr);
            c->resnorm_async(c->S[0]);
        }
        BLAUNCH(k_b_gather, dim3(((int)inst.size() + 127) / 128), dim3(128), 0, stream, scal_ptrs,
                (int)inst.size(), rel_dev);
        if (!preparing) IGAMG_HIP(hipGetLastError());
    }

    void run_round(const std::vector<int>& act, int q) {
        if (act != plan_active || q != plan_q) {
            clear_plan();
            preparing = true;
            restart_round(act, q);
            preparing = false;
            upload_plan();
            cursor = 0;
            IGAMG_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            try {
                restart_round(act, q);
            } catch (...) {
                hipGraph_t gg = nullptr;
                (void)hipStreamEndCapture(stream, &gg);
                if (gg) (void)hipGraphDestroy(gg);
                throw;
            }
            IGAMG_HIP(hipStreamEndCapture(stream, &graph));
            IGAMG_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
            plan_active = act;
            plan_q = q;
        }
        IGAMG_HIP(hipGraphLaunch(gexec, stream));
        destroy_retired();
        IGAMG_HIP(hipMemcpyAsync(rel_host, rel_dev, inst.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 stream));
        IGAMG_HIP(hipStreamSynchronize(stream));
    }
};

#undef BLAUNCH

// ---------------------------------------------------------------------------
// Scratch of igamg_extrap_coeffs_noalloc: one copy per GPU, held until the
// process ends.  Layout in doubles: the coefficient record (256 bytes), the
// leaf R factors of up to kNoAllocMaxN unknowns (one (q+1)^2 block per
// kQrRows-row panel, q <= kMaxQ), then the first tree level.  Every block a
// call reads was written earlier in the same call, so nothing is cleared.

namespace {

constexpr long long kNoAllocMaxN = 1LL << 23;
constexpr long long kNoAllocLeaves = kNoAllocMaxN / kQrRows;
constexpr long long kNoAllocNodes =
    (kNoAllocLeaves + kQrRows / kMaxCols - 1) / (kQrRows / kMaxCols);
constexpr size_t kScratchCoeffs = 32;
static_assert(sizeof(ExtrapCoeffs) <= kScratchCoeffs * sizeof(double), "coefficient record");
constexpr size_t kScratchDoubles =
    kScratchCoeffs + (size_t)(kNoAllocLeaves + kNoAllocNodes) * kMaxCols * kMaxCols;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch array, looked up once per device
// with that device current (in host code the array's name only stands in for
// it).  Called at context setup and, for a device with no context yet, by the
// first igamg_extrap_coeffs_noalloc call there.
double* scratch_for_current_device() {
    int dev = 0;
    IGAMG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        throw Error(IGAMG_EINVAL, "device index " + std::to_string(dev) + " beyond the scratch table");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        IGAMG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error(IGAMG_EHIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = (double*)ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

namespace {

template <class F>
igamg_status guarded(F&& f) {
    try {
        f();
        g_last_error.clear();
        return IGAMG_OK;
    } catch (const Error& e) {
        g_last_error = e.what();
        return (igamg_status)e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return IGAMG_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return IGAMG_EINVAL;
    }
}

void need(bool cond, const char* what) {
    if (!cond) throw Error(IGAMG_EINVAL, what);
}

}  // namespace

extern "C" {

void igamg_options_default(igamg_options* opt) {
    if (!opt) return;
    opt->nu1 = 2;
    opt->nu2 = 2;
    opt->smoother = IGAMG_SMOOTH_MCGS;
    opt->omega = 2.0 / 3.0;
    opt->precision = IGAMG_FP64;
    opt->n_el_coarsest = 4;
    opt->use_graphs = 1;
    opt->tail_items = 32;
    opt->stored_stencil = 0;
    opt->mu = 1;
    opt->pde = IGAMG_PDE_POISSON;
    opt->monitor = 0;
    opt->row_sweeps = 1;
    opt->stream = nullptr;
}

const char* igamg_last_error(void) { return g_last_error.c_str(); }

igamg_status igamg_setup(const igamg_geometry* geom, int degree, int levels,
                         const igamg_options* opt, igamg_ctx** out) {
    return guarded([&] {
        need(geom && out, "null argument");
        need(levels >= 0, "levels must be >= 0");
        *out = nullptr;
        std::unique_ptr<igamg_ctx> c(new igamg_ctx());
        if (opt)
            c->opt = *opt;
        else
            igamg_options_default(&c->opt);
        c->setup(*geom, degree, levels);
        (void)scratch_for_current_device();
        *out = c.release();
    });
}

void igamg_destroy(igamg_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
}

igamg_status igamg_ndof(const igamg_ctx* ctx, long long* n) {
    return guarded([&] {
        need(ctx && n, "null argument");
        *n = ctx->lv[ctx->L].N;
    });
}

igamg_status igamg_num_levels(const igamg_ctx* ctx, int* nlevels) {
    return guarded([&] {
        need(ctx && nlevels, "null argument");
        *nlevels = ctx->L + 1;
    });
}

igamg_status igamg_level_ndof(const igamg_ctx* ctx, int level, long long* n) {
    return guarded([&] {
        need(ctx && n, "null argument");
        need(level >= 0 && level <= ctx->L, "level out of range");
        *n = ctx->lv[level].N;
    });
}

igamg_status igamg_set_rhs(igamg_ctx* ctx, const double* bsrc, int on_device) {
    return guarded([&] {
        need(ctx && bsrc, "null argument");
        long long N = ctx->lv[ctx->L].N;
        IGAMG_HIP(hipMemcpyAsync(ctx->b, bsrc, N * sizeof(double),
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                 ctx->stream));
        double nb = ctx->vector_norm(ctx->b, N);
        if (!std::isfinite(nb)) throw Error(IGAMG_ENONFINITE, "right-hand side is not finite");
        ctx->set_bnorm(nb);
    });
}

igamg_status igamg_set_rhs_field(igamg_ctx* ctx, const double* modes, int n_modes) {
    return guarded([&] {
        need(ctx && modes && n_modes > 0, "bad mode table");
        ctx->set_rhs_field(modes, n_modes);
    });
}

igamg_status igamg_set_rhs_builtin(igamg_ctx* ctx) {
    return guarded([&] {
        need(ctx, "null argument");
        need(ctx->opt.pde != IGAMG_PDE_POISSON, "the Poisson operator has no built-in right-hand side");
        ctx->set_rhs_field(nullptr, -1);
    });
}

igamg_status igamg_get_rhs(igamg_ctx* ctx, double* b_dev) {
    return guarded([&] {
        need(ctx && b_dev, "null argument");
        ctx->copy(ctx->b, b_dev, ctx->lv[ctx->L].N);
        ctx->sync();
    });
}

igamg_status igamg_set_precision(igamg_ctx* ctx, int precision) {
    return guarded([&] {
        need(ctx, "null argument");
        need(precision == IGAMG_FP64 || precision == IGAMG_FP32_IR, "bad precision");
        if (precision != ctx->opt.precision) {
            ctx->opt.precision = precision;
            if (ctx->tail_auto) ctx->apply_cached_choice();  // the tuned shapes of this precision, if any
            ctx->choose_tail();      // the LDS store holds more FP32 levels
            ctx->graph_method = -1;  // recapture the restart cycle
        }
    });
}

igamg_status igamg_vcycle(igamg_ctx* ctx, double* x_dev) {
    return guarded([&] {
        need(ctx && x_dev, "null argument");
        ctx->G(x_dev);
        ctx->sync();
    });
}

igamg_status igamg_residual(igamg_ctx* ctx, const double* x_dev, double* rel) {
    return guarded([&] {
        need(ctx && x_dev && rel, "null argument");
        ctx->resnorm_async(x_dev);
        *rel = ctx->read_scal();
    });
}

igamg_status igamg_extrapolate(igamg_ctx* ctx, int method, int q, double* x_dev,
                               double* iterates_dev, double* gamma) {
    return guarded([&] {
        need(ctx && x_dev, "null argument");
        need(method == IGAMG_RRE || method == IGAMG_MPE, "method must be RRE or MPE");
        need(q >= 1 && q <= kMaxQ, "q must be in 1..8");
        ctx->ensure_iterates(q);
        long long N = ctx->lv[ctx->L].N;
        ctx->copy(x_dev, ctx->S[0], N);
        for (int j = 0; j <= q; ++j) {
            ctx->copy(ctx->S[j], ctx->S[j + 1], N);
            ctx->G(ctx->S[j + 1]);
        }
        if (iterates_dev)
            for (int j = 0; j <= q + 1; ++j) ctx->copy(ctx->S[j], iterates_dev + (size_t)j * N, N);
        IterPtrs it = ctx->iter_ptrs(q);
        ctx->extrap_coeffs_async(it, q, method);
        hipLaunchKernelGGL(k_extrap_combine, dim3(grid_for(N)), dim3(kBlock), 0, ctx->stream, it, q, N,
                           (const ExtrapCoeffs*)ctx->coeffs, x_dev, (double*)nullptr);
        ctx->check_launch();
        ExtrapCoeffs c = ctx->read_coeffs();
        if (gamma)
            for (int j = 0; j <= q; ++j) gamma[j] = c.gamma[j];
        if (c.info == -2) throw Error(IGAMG_ENONFINITE, "non-finite iterates");
        if (c.info == -1) throw Error(IGAMG_EBREAKDOWN, "extrapolation broke down (sum d = 0)");
    });
}

igamg_status igamg_generalized_residual(const igamg_ctx* ctx, double* gres) {
    return guarded([&] {
        need(ctx && gres, "null argument");
        need(ctx->have_coeffs, "no extrapolation yet");
        *gres = ctx->last_coeffs.gres;
    });
}

igamg_status igamg_solve(igamg_ctx* ctx, double tol, int max_restarts, int method, int q,
                         double* x_dev, igamg_stats* stats) {
    igamg_stats st{};
    auto t0 = std::chrono::steady_clock::now();
    bool converged = false;
    igamg_state rs{};
    bool resumed = false;
    igamg_status s = guarded([&] {
        need(ctx && x_dev, "null argument");
        resumed = ctx->resume;
        rs = ctx->resume_state;
        ctx->resume = false;  // a loaded state applies to this call only
        need(tol > 0 && max_restarts > 0, "bad tolerance or max_restarts");
        need(method == IGAMG_EXTRAP_NONE || method == IGAMG_RRE || method == IGAMG_MPE, "bad method");
        if (method != IGAMG_EXTRAP_NONE) need(q >= 1 && q <= kMaxQ, "q must be in 1..8");
        if (resumed)
            need(rs.method == method && (method == IGAMG_EXTRAP_NONE || rs.q == q),
                 "the loaded state belongs to another method or q");
        st.setup_ms = ctx->setup_ms;
        long long N = ctx->lv[ctx->L].N;
        // counters and adaptive settings carried over from a checkpoint
        double prev = 1.0;             // relative residual of the accepted iterate (x_0 = 0: 1)
        double d0_first = 0.0, ratio = -1.0;
        bool learned_off = false;
        if (resumed) {
            st.restarts = rs.restarts;
            st.vcycles = rs.vcycles;
            st.breakdowns = rs.breakdowns;
            st.learned_fallbacks = rs.learned_fallbacks;
            st.residual_checks = rs.residual_checks;
            st.rel_residual = rs.rel_residual;
            prev = rs.rel_residual;
            d0_first = rs.gen_scale;
            ratio = rs.monitor_ratio;
            learned_off = rs.learned_off != 0;
        }
        ctx->have_state = false;
        ctx->ensure_iterates(method == IGAMG_EXTRAP_NONE ? 0 : q);
        ctx->copy(x_dev, ctx->S[0], N);
        ctx->copy(x_dev, ctx->ckpt, N);
        const bool learned_at_start = ctx->learned_on;
        if (learned_off && ctx->learned_on) {
            ctx->learned_on = false;
            ctx->graph_method = -1;
        }
        // on every exit: x_dev (and the checkpoint) hold the accepted iterate,
        // the learned step is back as it was, the state is recorded
        auto finish = [&](bool finite) {
            if (finite) ctx->copy(ctx->S[0], ctx->ckpt, N);
            else ctx->copy(ctx->ckpt, ctx->S[0], N);
            ctx->copy(ctx->ckpt, x_dev, N);
            ctx->sync();
            igamg_state& o = ctx->state;
            o.method = method;
            o.q = method == IGAMG_EXTRAP_NONE ? 0 : q;
            o.restarts = st.restarts;
            o.vcycles = st.vcycles;
            o.breakdowns = st.breakdowns;
            o.learned_fallbacks = st.learned_fallbacks;
            o.residual_checks = st.residual_checks;
            o.learned_off = (learned_at_start && !ctx->learned_on) ? 1 : 0;
            o.rel_residual = st.rel_residual;
            o.gen_scale = d0_first;
            o.monitor_ratio = ratio;
            ctx->have_state = true;
            if (learned_at_start && !ctx->learned_on) {
                ctx->learned_on = true;  // the fallback lasts for this solve only
                ctx->graph_method = -1;
            }
        };
        // a non-finite cycle: the iterate it started from is the accepted one
        auto fail_nonfinite = [&](const char* what) {
            ctx->copy(ctx->ckpt, ctx->S[0], N);
            ctx->resnorm_async(ctx->S[0]);
            st.rel_residual = ctx->read_scal();
            finish(false);
            throw Error(IGAMG_ENONFINITE, what);
        };
        if (method == IGAMG_EXTRAP_NONE) {
            while (st.restarts < max_restarts) {
                ctx->run_restart_cycle(IGAMG_EXTRAP_NONE, 0);
                double rel = ctx->read_scal();
                if (!std::isfinite(rel)) fail_nonfinite("non-finite residual");
                st.vcycles++;
                st.restarts++;
                st.residual_checks++;
                st.rel_residual = rel;
                prev = rel;
                if (rel <= tol) {
                    converged = true;
                    break;
                }
            }
            finish(true);
        } else {
            // generalised-residual monitor: ||b - A t|| is evaluated when
            // ratio * g <= 4 tol, ratio = rel/g at the last evaluation
            const bool monitor = ctx->opt.monitor != 0;
            while (st.restarts < max_restarts) {
                const bool first = st.restarts == 0;
                ExtrapCoeffs c;
                double rel;
                if (!monitor) {
                    ctx->run_restart_cycle(method, q);
                    rel = ctx->read_cycle(c);
                    st.residual_checks++;
                } else {
                    ctx->run_restart_cycle(method, q, false);
                    c = ctx->read_coeffs();
                    if (first) d0_first = c.d0 > 0.0 ? c.d0 : 1.0;
                    const double g = c.gres / d0_first;
                    if (ratio < 0.0 || !std::isfinite(g) || ratio * g <= 4.0 * tol ||
                        st.restarts + 1 == max_restarts) {
                        ctx->resnorm_async(ctx->S[0]);
                        rel = ctx->read_scal();
                        st.residual_checks++;
                        if (std::isfinite(g) && g > 0.0) ratio = rel / g;
                    } else {
                        rel = ratio * g;  // estimate (above 4 tol): not converged
                    }
                }
                if (c.info == -2 || !std::isfinite(rel)) fail_nonfinite("non-finite iterate");
                if (std::isfinite(c.gres) && d0_first == 0.0 && c.d0 > 0.0) d0_first = c.d0;
                st.gen_residual = d0_first > 0.0 ? c.gres / d0_first : c.gres;
                // learned-smoother fallback: a cycle contracting worse than plain
                // V-cycles would (measured at training) switches back to Gauss-Seidel
                if (ctx->learned_on && ctx->rho_plain_ref > 0.0 && !first &&
                    rel / prev > std::pow(ctx->rho_plain_ref, q + 1) && rel > tol) {
                    ctx->learned_on = false;
                    ctx->graph_method = -1;
                    st.learned_fallbacks++;
                }
                prev = rel;
                st.vcycles += q + 1;
                st.restarts++;
                if (c.info == -1) st.breakdowns++;
                st.rel_residual = rel;
                if (rel <= tol) {
                    converged = true;
                    break;
                }
            }
            finish(true);
        }
        if (!converged) throw Error(IGAMG_ENOCONV, "tolerance not reached within max_restarts");
    });
    st.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return s;
}

igamg_status igamg_get_state(igamg_ctx* ctx, double* x_dev, igamg_state* state) {
    return guarded([&] {
        need(ctx && state, "null argument");
        need(ctx->have_state, "no restarted solve to checkpoint");
        if (x_dev) {
            ctx->copy(ctx->ckpt, x_dev, ctx->lv[ctx->L].N);
            ctx->sync();
        }
        *state = ctx->state;
    });
}

igamg_status igamg_set_state(igamg_ctx* ctx, const igamg_state* state) {
    return guarded([&] {
        need(ctx && state, "null argument");
        const igamg_state& r = *state;
        need(r.method == IGAMG_EXTRAP_NONE || r.method == IGAMG_RRE || r.method == IGAMG_MPE, "bad method");
        need(r.method == IGAMG_EXTRAP_NONE || (r.q >= 1 && r.q <= kMaxQ), "bad q");
        need(r.restarts >= 0 && r.vcycles >= 0 && r.breakdowns >= 0 && r.learned_fallbacks >= 0 &&
                 r.residual_checks >= 0, "negative counter");
        need(std::isfinite(r.rel_residual) && r.rel_residual >= 0.0, "bad rel_residual");
        need(std::isfinite(r.gen_scale) && std::isfinite(r.monitor_ratio), "bad monitor state");
        ctx->resume_state = r;
        ctx->resume = true;
    });
}

igamg_status igamg_solve_fgmres(igamg_ctx* ctx, double tol, int max_iters, int m, int precond, int q,
                                double* x_dev, igamg_stats* stats) {
    igamg_stats st{};
    auto t0 = std::chrono::steady_clock::now();
    igamg_status s = guarded([&] {
        need(ctx && x_dev, "null argument");
        need(tol > 0 && max_iters > 0, "bad tolerance or max_iters");
        need(m >= 1 && m <= kMaxKrylov, "restart length m must be in 1..30");
        need(precond == IGAMG_PRECOND_VCYCLE || precond == IGAMG_PRECOND_RRE || precond == IGAMG_PRECOND_MPE,
             "bad preconditioner");
        need(precond == IGAMG_PRECOND_VCYCLE || (q >= 1 && q <= kMaxQ), "q must be in 1..8");
        st.setup_ms = ctx->setup_ms;
        ctx->fgmres(tol, max_iters, m, precond, q, x_dev, st);
        ctx->sync();
    });
    st.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return s;
}

igamg_status igamg_get_operator_rows(igamg_ctx* ctx, int level, const long long* rows, int nrows,
                                     double* out) {
    return guarded([&] {
        need(ctx && rows && out && nrows >= 0, "null argument");
        need(level >= 0 && level <= ctx->L, "level out of range");
        Level& v = ctx->lv[level];
        int p = ctx->p, W = 2 * p + 1;
        int Sn = (ctx->dim == 2) ? W * W : W * W * W;
        for (int r = 0; r < nrows; ++r) need(rows[r] >= 0 && rows[r] < v.N, "row out of range");
        if (nrows == 0) return;
        if (ctx->kind == OP_STENCIL2D) {
            std::vector<long long> rv(rows, rows + nrows);
            long long* drows = ctx->upload(rv);
            double* dout = ctx->alloc<double>((size_t)nrows * Sn);
            ctx->with_p([&](auto PC) {
                constexpr int P = decltype(PC)::value;
                hipLaunchKernelGGL(k_gather_rows<P>, dim3(grid_for((long long)nrows * Sn)), dim3(kBlock),
                                   0, ctx->stream, v.coef64, v.n, v.ncp, drows, nrows, dout);
            });
            ctx->check_launch();
            IGAMG_HIP(hipMemcpyAsync(out, dout, (size_t)nrows * Sn * sizeof(double),
                                     hipMemcpyDeviceToHost, ctx->stream));
            ctx->sync();
            ctx->release(drows);
            ctx->release(dout);
            return;
        }
        int n = v.n;
        for (int r = 0; r < nrows; ++r) {
            long long I = rows[r];
            int i = (int)(I % n), j = (int)((I / n) % n), k = (ctx->dim == 3) ? (int)(I / ((long long)n * n)) : 0;
            for (int o = 0; o < Sn; ++o) {
                int di = o % W - p, dj = (o / W) % W - p, dk = (ctx->dim == 3) ? o / (W * W) - p : 0;
                double val = 0.0;
                if (i + di >= 0 && i + di < n && j + dj >= 0 && j + dj < n && k + dk >= 0 && k + dk < n) {
                    const Band1D &K = v.Kh, &M = v.Mh;
                    if (ctx->dim == 2)
                        val = K.at(i, di) * M.at(j, dj) + M.at(i, di) * K.at(j, dj);
                    else
                        val = K.at(i, di) * M.at(j, dj) * M.at(k, dk) +
                              M.at(i, di) * K.at(j, dj) * M.at(k, dk) +
                              M.at(i, di) * M.at(j, dj) * K.at(k, dk);
                }
                out[(size_t)r * Sn + o] = val;
            }
        }
    });
}

igamg_status igamg_apply(igamg_ctx* ctx, int level, const double* x_dev, double* y_dev) {
    return guarded([&] {
        need(ctx && x_dev && y_dev, "null argument");
        need(level >= 0 && level <= ctx->L, "level out of range");
        ctx->residual<double, double>(level, nullptr, x_dev, y_dev, 1, nullptr);
        ctx->sync();
    });
}

igamg_status igamg_smooth(igamg_ctx* ctx, int level, const double* b_dev, double* x_dev, int nsweeps) {
    return guarded([&] {
        need(ctx && b_dev && x_dev && nsweeps >= 0, "bad argument");
        need(level >= 1 && level <= ctx->L, "level out of range");
        ctx->smooth<double>(level, b_dev, x_dev, nsweeps);
        ctx->sync();
    });
}

igamg_status igamg_restrict(igamg_ctx* ctx, int level, const double* r_dev, double* rc_dev) {
    return guarded([&] {
        need(ctx && r_dev && rc_dev, "null argument");
        need(level >= 1 && level <= ctx->L, "level out of range");
        ctx->restrict_<double>(level, r_dev, rc_dev);
        ctx->sync();
    });
}

igamg_status igamg_prolong_add(igamg_ctx* ctx, int level, const double* e_dev, double* x_dev) {
    return guarded([&] {
        need(ctx && e_dev && x_dev, "null argument");
        need(level >= 1 && level <= ctx->L, "level out of range");
        ctx->prolong_<double>(level, e_dev, x_dev);
        ctx->sync();
    });
}

igamg_status igamg_coarse_solve(igamg_ctx* ctx, const double* b_dev, double* x_dev) {
    return guarded([&] {
        need(ctx && b_dev && x_dev, "null argument");
        ctx->coarse<double>(b_dev, x_dev);
        ctx->sync();
    });
}

igamg_status igamg_extrap_coeffs(igamg_ctx* ctx, int method, int q, const double* iterates_dev,
                                 double* gamma, int* info) {
    return guarded([&] {
        need(ctx && iterates_dev && gamma, "null argument");
        need(method == IGAMG_RRE || method == IGAMG_MPE, "method must be RRE or MPE");
        need(q >= 1 && q <= kMaxQ, "q must be in 1..8");
        ctx->ensure_iterates(q);
        long long N = ctx->lv[ctx->L].N;
        IterPtrs it{};
        for (int j = 0; j <= q + 1; ++j) it.s[j] = iterates_dev + (size_t)j * N;
        ctx->extrap_coeffs_async(it, q, method);
        ExtrapCoeffs c = ctx->read_coeffs();
        for (int j = 0; j <= q; ++j) gamma[j] = c.gamma[j];
        if (info) *info = c.info;
    });
}

igamg_status igamg_extrap_coeffs_noalloc(igamg_ctx* ctx, int method, int q, const double* iterates_dev,
                                         double* gamma, int* info) {
    return guarded([&] {
        need(ctx && iterates_dev && gamma, "null argument");
        need(method == IGAMG_RRE || method == IGAMG_MPE, "method must be RRE or MPE");
        need(q >= 1 && q <= kMaxQ, "q must be in 1..8");
        const long long N = ctx->lv[ctx->L].N;
        if (N > kNoAllocMaxN)
            throw Error(IGAMG_EINVAL, "igamg_extrap_coeffs_noalloc: " + std::to_string(N) +
                                          " unknowns exceed its scratch limit of " +
                                          std::to_string(kNoAllocMaxN));
        double* sc = scratch_for_current_device();
        ExtrapCoeffs* cf = reinterpret_cast<ExtrapCoeffs*>(sc);
        double* R0 = sc + kScratchCoeffs;
        double* R1 = R0 + (size_t)kNoAllocLeaves * kMaxCols * kMaxCols;
        IterPtrs it{};
        for (int j = 0; j <= q + 1; ++j) it.s[j] = iterates_dev + (size_t)j * N;
        tsqr_coeffs_async(ctx->stream, it, q, N, method, R0, R1, cf);
        IGAMG_HIP(hipMemcpyAsync(ctx->host_coeffs, cf, sizeof(ExtrapCoeffs), hipMemcpyDeviceToHost,
                                 ctx->stream));
        IGAMG_HIP(hipStreamSynchronize(ctx->stream));
        const ExtrapCoeffs c = *ctx->host_coeffs;
        ctx->last_coeffs = c;
        ctx->have_coeffs = true;
        for (int j = 0; j <= q; ++j) gamma[j] = c.gamma[j];
        if (info) *info = c.info;
    });
}

igamg_status igamg_profile_smoother(igamg_ctx* ctx, int level, int precision, int nsweeps,
                                    double* avg_ms, double* bytes, int* launches) {
    return guarded([&] {
        need(ctx && avg_ms && bytes && launches && nsweeps > 0, "bad argument");
        need(level >= 1 && level <= ctx->L, "level out of range");
        need(precision == IGAMG_FP64 || precision == IGAMG_FP32_IR, "bad precision");
        ctx->profile_smoother(level, precision, nsweeps, avg_ms, bytes, launches);
    });
}

igamg_status igamg_setup_batch(int count, const igamg_geometry* geoms, const int* degrees,
                               const igamg_options* opt, igamg_batch** out) {
    return guarded([&] {
        need(count >= 1 && geoms && degrees && out, "bad argument");
        *out = nullptr;
        std::unique_ptr<igamg_batch> B(new igamg_batch());
        igamg_options o;
        if (opt)
            o = *opt;
        else
            igamg_options_default(&o);
        need(o.mu == 1, "batched solves run V-cycles (mu = 1)");
        need(o.pde == IGAMG_PDE_POISSON, "batched solves take the Poisson operator");
        if (o.stream) {
            B->stream = (hipStream_t)o.stream;
        } else {
            IGAMG_HIP(hipStreamCreateWithFlags(&B->stream, hipStreamDefault));
            B->own_stream = true;
        }
        o.stream = B->stream;
        o.precision = IGAMG_FP32_IR;
        o.smoother = IGAMG_SMOOTH_MCGS;
        o.stored_stencil = 1;
        if (!opt) o.tail_items = 32;
        const bool tune = o.tail_items < 0;
        o.n_el_coarsest = 0;
        o.use_graphs = 0;
        for (int i = 0; i < count; ++i) {
            need(geoms[i].kind == IGAMG_UNIT_SQUARE || geoms[i].kind == IGAMG_QUARTER_ANNULUS,
                 "batches hold 2D problems");
            std::unique_ptr<igamg_ctx> c(new igamg_ctx());
            c->opt = o;
            c->setup(geoms[i], degrees[i], 0);
            if (tune) {
                bool cached;
                {
                    std::lock_guard<std::mutex> g(g_tune_mu);
                    cached = g_tune_cache.count(c->tune_key()) > 0;
                }
                if (!cached) c->autotune(nullptr, nullptr, false);  // batches have no learned step
            }
            B->inst.push_back(c.release());
        }
        for (int g = 0; g < 5; ++g) {
            hipStream_t st;
            IGAMG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            B->side.push_back(st);
        }
        for (int e = 0; e < 6; ++e) {
            hipEvent_t evv;
            IGAMG_HIP(hipEventCreateWithFlags(&evv, hipEventDisableTiming));
            B->ev.push_back(evv);
        }
        IGAMG_HIP(hipMalloc((void**)&B->rel_dev, count * sizeof(double)));
        IGAMG_HIP(hipHostMalloc((void**)&B->rel_host, count * sizeof(double), hipHostMallocDefault));
        std::vector<const double*> sp(count);
        for (int i = 0; i < count; ++i) sp[i] = B->inst[i]->scal;
        IGAMG_HIP(hipMalloc((void**)&B->scal_ptrs, count * sizeof(double*)));
        IGAMG_HIP(hipMemcpy((void*)B->scal_ptrs, sp.data(), count * sizeof(double*), hipMemcpyHostToDevice));
        *out = B.release();
    });
}

void igamg_destroy_batch(igamg_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
}

igamg_status igamg_batch_instance(igamg_batch* b, int i, igamg_ctx** ctx) {
    return guarded([&] {
        need(b && ctx && i >= 0 && i < (int)b->inst.size(), "bad argument");
        *ctx = b->inst[i];
    });
}

igamg_status igamg_solve_batch(igamg_batch* b, double tol, int max_restarts, int q,
                               double* const* x_dev, igamg_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    int n = b ? (int)b->inst.size() : 0;
    std::vector<igamg_stats> st(n);
    bool all = false;
    igamg_status s = guarded([&] {
        need(b && x_dev && tol > 0 && max_restarts > 0, "bad argument");
        need(q >= 1 && q <= kMaxQ, "q must be in 1..8");
        std::vector<int> act;
        for (int i = 0; i < n; ++i) {
            need(x_dev[i] != nullptr, "null iterate");
            igamg_ctx* c = b->inst[i];
            c->ensure_iterates(q);
            c->copy(x_dev[i], c->S[0], c->lv[c->L].N);
            act.push_back(i);
        }
        for (int k = 0; k < max_restarts && !act.empty(); ++k) {
            b->run_round(act, q);
            std::vector<int> next;
            for (int i : act) {
                double rel = b->rel_host[i];
                st[i].restarts++;
                st[i].vcycles += q + 1;
                st[i].rel_residual = rel;
                if (!std::isfinite(rel)) throw Error(IGAMG_ENONFINITE, "non-finite residual in a batch problem");
                if (rel > tol) next.push_back(i);
            }
            act = next;
        }
        for (int i = 0; i < n; ++i) {
            igamg_ctx* c = b->inst[i];
            c->copy(c->S[0], x_dev[i], c->lv[c->L].N);
            st[i].setup_ms = c->setup_ms;
        }
        IGAMG_HIP(hipStreamSynchronize(b->stream));
        all = act.empty();
        if (!all) throw Error(IGAMG_ENOCONV, "some batch problems did not converge");
    });
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats)
        for (int i = 0; i < n; ++i) {
            st[i].solve_ms = ms;
            stats[i] = st[i];
        }
    return s;
}

igamg_status igamg_autotune(igamg_ctx* ctx, int* tail_items, double* vcycle_ms) {
    return guarded([&] {
        need(ctx, "null argument");
        ctx->autotune(tail_items, vcycle_ms);
    });
}

igamg_status igamg_get_tuning(const igamg_ctx* ctx, igamg_tuning* out) {
    return guarded([&] {
        need(ctx && out, "null argument");
        need(ctx->L + 1 <= 16, "more levels than the report holds");
        *out = igamg_tuning{};
        out->tail_items = ctx->opt.tail_items;
        out->tail_top = ctx->tail_top;
        out->num_levels = ctx->L + 1;
        for (int l = 0; l <= ctx->L; ++l) {
            out->row_class[l] = ctx->sweep_shape(l);
            out->learned_kernel[l] = ctx->learned_kern[l];
        }
        out->vcycle_ms = ctx->tuned_ms;
    });
}

igamg_status igamg_set_tuning(igamg_ctx* ctx, const igamg_tuning* in) {
    return guarded([&] {
        need(ctx && in, "null argument");
        need(in->num_levels == ctx->L + 1, "num_levels does not match the hierarchy");
        need(in->tail_items >= 0, "tail_items must be >= 0");
        for (int l = 0; l <= ctx->L; ++l) {
            need(in->row_class[l] >= 0 && in->row_class[l] <= (ctx->kind == OP_KRON3D ? 2 : 1),
                 "row_class must be 0 or 1 (cubes: 0, 1 or 2)");
            const int k = in->learned_kernel[l];
            need(k == 0 || k == 12 || k == 28 || k == 29, "learned_kernel must be 0, 12, 28 or 29");
        }
        for (int l = 0; l <= ctx->L; ++l) {
            ctx->row_pref[l] = in->row_class[l];
            ctx->learned_kern[l] = in->learned_kernel[l];
        }
        ctx->opt.tail_items = in->tail_items;
        ctx->tail_auto = false;
        ctx->choose_tail();
        ctx->graph_method = -1;
    });
}

void igamg_train_options_default(igamg_train_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->vcycles_per_rhs = 3;
    o->epochs = 10;
    o->batch = 32;
    o->lr = 1e-3;
    o->seed = 5000;
    o->val_vcycles = 12;
    o->solve_tol = 1e-12;
}

igamg_status igamg_train_smoother(igamg_ctx* ctx, const igamg_train_options* o,
                                  igamg_train_report* report) {
    return guarded([&] {
        need(ctx && o, "null argument");
        need(ctx->opt.mu == 1, "the smoother is trained on V-cycles (mu = 1)");
        need(ctx->opt.pde == IGAMG_PDE_POISSON, "the smoother is trained for the Poisson operator");
        igamg_train_report rep{};
        ctx->train(*o, rep);
        if (report) *report = rep;
    });
}

igamg_status igamg_set_learned(igamg_ctx* ctx, int enabled) {
    return guarded([&] {
        need(ctx, "null argument");
        bool any = false;
        for (auto& n : ctx->nets) any = any || n.have;
        need(!enabled || any, "no learned smoother weights loaded");
        ctx->learned_on = enabled != 0;
        ctx->graph_method = -1;
    });
}

igamg_status igamg_get_smoother_weights(igamg_ctx* ctx, int level, uint16_t* w, size_t n) {
    return guarded([&] {
        need(ctx && w && n == (size_t)kLWeights, "need 2592 values");
        need(level >= 1 && level <= ctx->L && level < (int)ctx->nets.size() && ctx->nets[level].have,
             "no weights on this level");
        IGAMG_HIP(hipMemcpyAsync(w, ctx->nets[level].wc, kLWeights * 2, hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
    });
}

igamg_status igamg_set_smoother_weights(igamg_ctx* ctx, int level, const uint16_t* w, size_t n) {
    return guarded([&] {
        need(ctx && w && n == (size_t)kLWeights, "need 2592 values");
        need(ctx->dim == 2, "the learned smoother is 2D only");
        need(level >= 1 && level <= ctx->L, "level out of range");
        ctx->ensure_net(level);
        auto& net = ctx->nets[level];
        IGAMG_HIP(hipMemcpyAsync(net.wc, w, kLWeights * 2, hipMemcpyHostToDevice, ctx->stream));
        std::vector<float> mw(kLWeights);
        for (int k = 0; k < kLWeights; ++k) {
            uint32_t u = ((uint32_t)w[k]) << 16;
            std::memcpy(&mw[k], &u, 4);
        }
        IGAMG_HIP(hipMemcpyAsync(net.master, mw.data(), kLWeights * 4, hipMemcpyHostToDevice, ctx->stream));
        hipLaunchKernelGGL(k_learned_layouts, dim3((kLWeights + 255) / 256), dim3(256), 0, ctx->stream,
                           (const uint16_t*)net.wc, net.w2f, net.w2b, net.mf32, net.mfbf);
        ctx->check_launch();
        ctx->sync();
        net.have = true;
        net.on = true;
        ctx->graph_method = -1;
    });
}

igamg_status igamg_smoother_forward(igamg_ctx* ctx, int level, const float* z, float* y) {
    return guarded([&] {
        need(ctx && z && y, "null argument");
        need(level >= 1 && level <= ctx->L && level < (int)ctx->nets.size() && ctx->nets[level].have,
             "no weights on this level");
        auto& v = ctx->lv[level];
        auto& net = ctx->nets[level];
        LImage im{z, v.n, v.n, v.n, 0, 0};
        (void)net;
        ctx->learned_apply<float>(level, im, nullptr, (float*)nullptr, y);
        ctx->sync();
    });
}

igamg_status igamg_smoother_loss_grad(igamg_ctx* ctx, int level, const float* z, const float* t,
                                      double* loss, float* grad) {
    return guarded([&] {
        need(ctx && z && t && loss && grad, "null argument");
        need(level >= 1 && level <= ctx->L && level < (int)ctx->nets.size() && ctx->nets[level].have,
             "no weights on this level");
        auto& v = ctx->lv[level];
        auto& net = ctx->nets[level];
        LItem it{LImage{z, v.n, v.n, v.n, 0, 0}, t, 0, v.n};
        LItem* dit = ctx->alloc<LItem>(1);
        IGAMG_HIP(hipMemcpyAsync(dit, &it, sizeof(LItem), hipMemcpyHostToDevice, ctx->stream));
        int tpr = (v.n + kLTile - 1) / kLTile, tiles = tpr * tpr;
        float* gpart = ctx->alloc<float>((size_t)tiles * kLWeights);
        double* lpart = ctx->alloc<double>(tiles);
        float* g = ctx->alloc<float>(kLWeights);
        double* ls = ctx->alloc<double>(1);
        LearnedW W{net.wc, net.w2f, net.w2b};
        hipLaunchKernelGGL(k_learned_train, dim3(tiles), dim3(kLThreads), 0, ctx->stream, (const LItem*)dit,
                           tiles, W, (float)(1.0 / ((double)v.N)), gpart, lpart);
        hipLaunchKernelGGL(k_learned_reduce, dim3((kLWeights + 255) / 256), dim3(256), 0, ctx->stream,
                           (const float*)gpart, tiles, (const double*)lpart, g, ls);
        ctx->check_launch();
        IGAMG_HIP(hipMemcpyAsync(grad, g, kLWeights * 4, hipMemcpyDeviceToHost, ctx->stream));
        IGAMG_HIP(hipMemcpyAsync(ctx->host_scal + 5, ls, 8, hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
        *loss = ctx->host_scal[5] / (double)v.N;
        for (void* a : {(void*)dit, (void*)gpart, (void*)lpart, (void*)g, (void*)ls}) ctx->release(a);
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// 1D model problems (Section 2.4): one workgroup per problem, one launch per call

struct igamg_set1d {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<igamg_problem1d> prob;
    std::vector<Desc1D> desc;
    std::vector<void*> mem;
    Desc1D* d_desc = nullptr;
    double** d_x = nullptr;
    Out1D* d_out = nullptr;
    Out1D* h_out = nullptr;

    template <typename T>
    T* alloc(size_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
            throw Error(IGAMG_ENOMEM, "device allocation failed");
        mem.push_back(p);
        return (T*)p;
    }
    template <typename T>
    T* upload(const std::vector<T>& v) {
        T* d = alloc<T>(v.size());
        IGAMG_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return d;
    }
    ~igamg_set1d() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (void* p : mem) (void)hipFree(p);
        if (h_out) (void)hipHostFree(h_out);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    // x_dev[i] of every problem, then one launch of k_solve1d
    void run(int mode, int iters, double tol, double* const* x_dev) {
        const int count = (int)prob.size();
        for (int i = 0; i < count; ++i) need(x_dev[i] != nullptr, "null iterate");
        IGAMG_HIP(hipMemcpyAsync(d_x, x_dev, count * sizeof(double*), hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(k_solve1d, dim3(count), dim3(kBlock), 0, stream, (const Desc1D*)d_desc,
                           (double* const*)d_x, mode, iters, tol, d_out);
        IGAMG_HIP(hipGetLastError());
        IGAMG_HIP(hipMemcpyAsync(h_out, d_out, count * sizeof(Out1D), hipMemcpyDeviceToHost, stream));
        IGAMG_HIP(hipStreamSynchronize(stream));
    }
};

namespace {

void setup_problem1d(igamg_set1d& S, const igamg_problem1d& pr, Desc1D& D) {
    const int p = pr.degree, ne = pr.n_el, nlev = pr.levels;
    need(p >= 1 && p <= kMax1DDegree, "1D degree must be in 1..9");
    need(nlev >= 1 && nlev <= kMax1DLevels, "1D levels must be in 1..16");
    need(ne >= 1 && ne <= (1 << 20), "1D n_el out of range");
    const int ne0 = ne >> (nlev - 1);
    need(ne0 >= 1 && (ne0 << (nlev - 1)) == ne, "n_el must be a multiple of 2^(levels-1)");
    need(pr.smoother == IGAMG_SMOOTH_JACOBI || pr.smoother == IGAMG_SMOOTH_MCGS ||
             pr.smoother == IGAMG_SMOOTH_LEXGS,
         "1D smoother must be weighted Jacobi or multicolour or lexicographic Gauss-Seidel");
    need(pr.nu1 >= 0 && pr.nu2 >= 0 && pr.nu1 <= 64 && pr.nu2 <= 64, "sweep counts must be in 0..64");
    need(pr.mu >= 1 && pr.mu <= kMaxMu, "mu must be in 1..4");
    need(pr.method == IGAMG_EXTRAP_NONE || pr.method == IGAMG_RRE || pr.method == IGAMG_MPE, "bad method");
    need(pr.method == IGAMG_EXTRAP_NONE || (pr.q >= 1 && pr.q <= kMaxQ), "q must be in 1..8");
    need(pr.omega > 0.0 && pr.omega < 2.0, "omega must be in (0, 2)");
    D = Desc1D{};
    D.p = p;
    D.L = nlev - 1;
    D.n_el = ne;
    D.nq = p + 1;
    D.smoother = pr.smoother;
    D.nu1 = pr.nu1;
    D.nu2 = pr.nu2;
    D.mu = pr.mu;
    D.method = pr.method;
    D.q = pr.method == IGAMG_EXTRAP_NONE ? 1 : pr.q;
    D.omega = pr.omega;
    long long lds = 0;
    for (int l = 0; l < nlev; ++l) {
        D.n[l] = (ne0 << l) + p - 2;
        need(D.n[l] >= 1, "a level has no interior unknowns");
        D.off[l] = (int)lds;
        lds += 3LL * D.n[l];
    }
    need(lds <= kLds1D, "1D problem too large for one workgroup's LDS");
    // the bands follow the vectors in LDS when they fit (read at LDS latency
    // by every step of the cycle), else they are read through the caches
    long long band_vals = 0;
    for (int l = 0; l < nlev; ++l) band_vals += (2LL * p + 1) * D.n[l];
    D.bands_lds = lds + band_vals <= kLds1D ? 1 : 0;
    for (int l = 0; l < nlev && D.bands_lds; ++l) {
        D.boff[l] = (int)lds;
        lds += (2LL * p + 1) * D.n[l];
    }
    // finest band by quadrature, coarser ones by the Galerkin product (eq. (4))
    std::vector<Band1D> K(nlev);
    Band1D M;
    stiffness_mass_bands(ne, p, K[D.L], M);
    for (int l = D.L; l >= 1; --l) {
        TransferTables T = transfer_tables(prolongation_boehm(ne0 << (l - 1), p));
        if (T.nf != D.n[l] || T.nc != D.n[l - 1]) throw Error(IGAMG_EINVAL, "transfer size mismatch");
        K[l - 1] = galerkin_band(K[l], T, p);
        D.rs[l] = S.upload(T.r_start);
        D.rw[l] = S.upload(T.r_w);
        D.RW[l] = T.RW;
        D.ps[l] = S.upload(T.p_start);
        D.pw[l] = S.upload(T.p_w);
        D.PW[l] = T.PW;
    }
    for (int l = 0; l < nlev; ++l) D.K[l] = S.upload(K[l].v);
    // coarsest inverse from the Cholesky factor
    const int n0 = D.n[0], W = 2 * p + 1;
    std::vector<double> A((size_t)n0 * n0, 0.0);
    for (int i = 0; i < n0; ++i)
        for (int d = -p; d <= p; ++d)
            if (i + d >= 0 && i + d < n0) A[(size_t)i * n0 + i + d] = K[0].v[(size_t)i * W + d + p];
    std::vector<double> inv;
    if (coarse_inverse(std::move(A), n0, true, inv) != 0)
        throw Error(IGAMG_ENOTSPD, "coarsest 1D operator is not SPD");
    D.Ainv0 = S.upload(inv);
    ElementTables E = element_tables(ne, p, p + 1);
    D.V = S.upload(E.V);
    D.wq = S.upload(E.wts);
    D.xq = S.upload(E.pts);
    const int nL = D.n[D.L];
    double* b = S.alloc<double>(nL);
    hipLaunchKernelGGL(k_load1d, dim3((nL + kBlock - 1) / kBlock), dim3(kBlock), 0, S.stream, ne, p, p + 1,
                       D.V, D.wq, D.xq, b);
    IGAMG_HIP(hipGetLastError());
    D.b = b;
    D.S = S.alloc<double>((size_t)(D.q + 2) * nL);
    D.Qm = S.alloc<double>((size_t)(D.q + 1) * nL);
}

igamg_set1d* checked_set(igamg_set1d* s, int i) {
    need(s != nullptr, "null set");
    need(i >= 0 && i < (int)s->prob.size(), "problem index out of range");
    return s;
}

}  // namespace

extern "C" {

void igamg_problem1d_default(igamg_problem1d* pr) {
    if (!pr) return;
    pr->n_el = 64;
    pr->degree = 2;
    pr->levels = 4;
    pr->smoother = IGAMG_SMOOTH_JACOBI;
    pr->nu1 = 1;
    pr->nu2 = 1;
    pr->mu = 1;
    pr->omega = 2.0 / 3.0;
    pr->method = IGAMG_EXTRAP_NONE;
    pr->q = 4;
}

igamg_status igamg_setup_1d(int count, const igamg_problem1d* probs, void* stream, igamg_set1d** out) {
    return guarded([&] {
        need(count >= 1 && probs && out, "bad argument");
        *out = nullptr;
        std::unique_ptr<igamg_set1d> S(new igamg_set1d());
        if (stream) {
            S->stream = (hipStream_t)stream;
        } else {
            IGAMG_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamDefault));
            S->own_stream = true;
        }
        S->prob.assign(probs, probs + count);
        S->desc.resize(count);
        for (int i = 0; i < count; ++i) setup_problem1d(*S, probs[i], S->desc[i]);
        S->d_desc = S->upload(S->desc);
        S->d_x = S->alloc<double*>(count);
        S->d_out = S->alloc<Out1D>(count);
        IGAMG_HIP(hipHostMalloc((void**)&S->h_out, count * sizeof(Out1D), hipHostMallocDefault));
        IGAMG_HIP(hipStreamSynchronize(S->stream));
        *out = S.release();
    });
}

void igamg_destroy_1d(igamg_set1d* set) { delete set; }

long long igamg_ndof_1d(const igamg_set1d* set, int i) {
    if (!set || i < 0 || i >= (int)set->prob.size()) return -1;
    return set->desc[i].n[set->desc[i].L];
}

igamg_status igamg_set_rhs_1d(igamg_set1d* set, int i, const double* b_dev) {
    return guarded([&] {
        checked_set(set, i);
        need(b_dev != nullptr, "null argument");
        const Desc1D& D = set->desc[i];
        IGAMG_HIP(hipMemcpyAsync((void*)D.b, b_dev, D.n[D.L] * sizeof(double), hipMemcpyDeviceToDevice,
                                 set->stream));
        IGAMG_HIP(hipStreamSynchronize(set->stream));
    });
}

igamg_status igamg_get_rhs_1d(igamg_set1d* set, int i, double* b_dev) {
    return guarded([&] {
        checked_set(set, i);
        need(b_dev != nullptr, "null argument");
        const Desc1D& D = set->desc[i];
        IGAMG_HIP(hipMemcpyAsync(b_dev, D.b, D.n[D.L] * sizeof(double), hipMemcpyDeviceToDevice, set->stream));
        IGAMG_HIP(hipStreamSynchronize(set->stream));
    });
}

igamg_status igamg_cycles_1d(igamg_set1d* set, int ncycles, double* const* x_dev) {
    return guarded([&] {
        need(set && x_dev && ncycles >= 0, "bad argument");
        set->run(1, ncycles, 0.0, x_dev);
    });
}

igamg_status igamg_solve_1d(igamg_set1d* set, double tol, int max_iters, double* const* x_dev,
                            igamg_stats1d* stats) {
    auto t0 = std::chrono::steady_clock::now();
    bool all = false;
    igamg_status s = guarded([&] {
        need(set && x_dev && tol > 0 && max_iters > 0, "bad argument");
        set->run(0, max_iters, tol, x_dev);
        all = true;
        for (size_t i = 0; i < set->prob.size(); ++i) {
            const Out1D& o = set->h_out[i];
            if (o.status != 0) throw Error(o.status, "non-finite values in a 1D solve");
            if (!o.converged) all = false;
        }
        if (!all) throw Error(IGAMG_ENOCONV, "some 1D problems did not converge");
    });
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats && set && (s == IGAMG_OK || s == IGAMG_ENOCONV || s == IGAMG_ENONFINITE)) {
        for (size_t i = 0; i < set->prob.size(); ++i) {
            const Out1D& o = set->h_out[i];
            stats[i] = igamg_stats1d{o.restarts, o.vcycles, o.breakdowns, o.converged, o.rel_residual, o.l2_error, ms};
        }
    }
    return s;
}

}  // extern "C"
