// Streaming copies used as practical HBM ceilings that the step kernels are
// compared against: flat copies (read `bytes`, write `bytes`), and the step's
// own access pattern without its arithmetic (every plane read at the pull
// source of its direction, written at the node).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm.h"
#include "../../include/lbm_probe.h"
#include "kernels.hpp"

namespace lbe {

// The pull pattern of a periodic node launch: the same addressing (Pull),
// block shape and non-temporal stores as the step kernel, no collision.
template <class L, class T>
__global__ void __launch_bounds__(BX)
k_pull_pattern(const T* __restrict__ src, T* __restrict__ dst, Grid g) {
    const NodePos pos = node_of_thread(g);
    if (!pos.in) return;
    const Pull<XBC_PERIODIC> pl(g, pos);
    T v[L::Q];
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        v[i] = ldp<L::Q>(src, i, pl.template src<L, i>());
    });
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        stp_nt<L::Q>(dst, i, pos.n, v[i]);
    });
}

typedef float v4f __attribute__((ext_vector_type(4)));

// mode 0: grid-stride loop, four independent 16-byte loads per thread per
//         iteration, non-temporal stores
// mode 1: one 16-byte element per thread, one-shot grid, non-temporal stores
// mode 2: as mode 1 with ordinary stores
__global__ void __launch_bounds__(256)
k_copy_ilp4(const v4f* __restrict__ src, v4f* __restrict__ dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v4f a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                     d = src[i + 3 * stride];
        __builtin_nontemporal_store(a, &dst[i]);
        __builtin_nontemporal_store(b, &dst[i + stride]);
        __builtin_nontemporal_store(c, &dst[i + 2 * stride]);
        __builtin_nontemporal_store(d, &dst[i + 3 * stride]);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(src[i], &dst[i]);
}

template <bool NT>
__global__ void __launch_bounds__(256)
k_copy_flat(const v4f* __restrict__ src, v4f* __restrict__ dst, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (NT) __builtin_nontemporal_store(src[i], &dst[i]);
    else dst[i] = src[i];
}

// The adjoint step's access pattern without its arithmetic: the forward
// state read at the pull source of each direction, the adjoint read at the
// node that pulls from this one (x + e_i), the result written at the node.
template <class L, class T>
__global__ void __launch_bounds__(BX)
k_adjoint_pattern(const T* __restrict__ fsrc, const T* __restrict__ lsrc, T* __restrict__ dst,
                  Grid g) {
    const NodePos pos = node_of_thread(g);
    if (!pos.in) return;
    const Pull<XBC_PERIODIC> pl(g, pos);
    T f[L::Q], lg[L::Q];
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        f[i] = ldp<L::Q>(fsrc, i, pl.template src<L, i>());
    });
    // x + e_i is the pull source of the opposite direction
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        lg[i] = ldp<L::Q>(lsrc, i, pl.template src<L, TAB<L>.opp[i]>());
    });
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        stp_nt<L::Q>(dst, i, pos.n, f[i] + lg[i]);
    });
}

// The pull pattern in a blocked layout: consecutive blocks of 2^lb nodes,
// each holding its Q planes one after the other (element (i, n) at
// (n >> lb) * (Q << lb) + (i << lb) + (n & (2^lb - 1))); otherwise as
// k_pull_pattern.
template <class L, class T>
__global__ void __launch_bounds__(BX)
k_blocked_pull_pattern(const T* __restrict__ src, T* __restrict__ dst, Grid g, uint32_t lb) {
    const NodePos pos = node_of_thread(g);
    if (!pos.in) return;
    const Pull<XBC_PERIODIC> pl(g, pos);
    const uint32_t mask = (1u << lb) - 1u;
    auto at = [&](uint32_t i, uint32_t n) {
        return (n >> lb) * ((uint32_t)L::Q << lb) + (i << lb) + (n & mask);
    };
    T v[L::Q];
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        v[i] = ld(src, at(i, pl.template src<L, i>()));
    });
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        st_nt(dst, at(i, pos.n), v[i]);
    });
}

// The in-place "AA" access pattern, one buffer, no arithmetic.  Even pass:
// node x reads every plane at x and writes plane i's value into plane ibar at
// x (node-local).  Odd pass: node x reads plane ibar at x - e_i and writes
// plane i at x + e_i.  In the odd pass the location (j, y) is read and
// written by the same node, y - e_j, so the pass is race-free in place.
template <class L, class T, bool ODD>
__global__ void __launch_bounds__(BX)
k_aa_pattern(T* buf, Grid g) {
    const NodePos pos = node_of_thread(g);
    if (!pos.in) return;
    const Pull<XBC_PERIODIC> pl(g, pos);
    T v[L::Q];
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ib = TAB<L>.opp[i];
        if constexpr (ODD) v[i] = ld(buf + (size_t)ib * g.S, pl.template src<L, i>());
        else v[i] = ld(buf + (size_t)i * g.S, pos.n);
    });
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ib = TAB<L>.opp[i];
        if constexpr (ODD) st_nt(buf + (size_t)i * g.S, pl.template src<L, ib>(), v[i]);
        else st_nt(buf + (size_t)ib * g.S, pos.n, v[i]);
    });
}

}  // namespace lbe

extern "C" int lbm_stream_copy(void* dst, const void* src, int64_t bytes, int32_t mode,
                               int32_t reps, double* ms_per_copy) {
    if (!dst || !src || bytes <= 0 || bytes % 16 != 0 || reps < 1 || mode < 0 || mode > 2)
        return LBM_EINVAL;
    const uint64_t n = (uint64_t)bytes / 16;
    hipStream_t s;
    hipEvent_t e0, e1;
    if (hipStreamCreate(&s) != hipSuccess) return LBM_EDEVICE;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return LBM_EDEVICE;
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
    const unsigned flat_blocks = (unsigned)((n + 255) / 256);
    const unsigned ilp_blocks = (unsigned)cus * 16u;
    auto launch = [&]() {
        if (mode == 0)
            hipLaunchKernelGGL(lbe::k_copy_ilp4, dim3(ilp_blocks), dim3(256), 0, s,
                               (const lbe::v4f*)src, (lbe::v4f*)dst, n);
        else if (mode == 1)
            hipLaunchKernelGGL(lbe::k_copy_flat<true>, dim3(flat_blocks), dim3(256), 0, s,
                               (const lbe::v4f*)src, (lbe::v4f*)dst, n);
        else
            hipLaunchKernelGGL(lbe::k_copy_flat<false>, dim3(flat_blocks), dim3(256), 0, s,
                               (const lbe::v4f*)src, (lbe::v4f*)dst, n);
    };
    launch();   // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(e1, s);
    int rc = LBM_OK;
    if (hipEventSynchronize(e1) != hipSuccess) rc = LBM_EDEVICE;
    float ms = 0.f;
    if (rc == LBM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = LBM_EDEVICE;
    if (ms_per_copy) *ms_per_copy = ms / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return rc;
}

namespace {

int pattern_copy(int lattice, int precision, void* dst, const void* src, const void* src2,
                 int64_t nx, int64_t ny, int64_t nz, int32_t reps, double* ms_per_copy) {
    if (!dst || !src || nx < 1 || ny < 1 || nz < 1 || reps < 1) return LBM_EINVAL;
    if (lattice < 0 || lattice > 2 || (precision != LBM_FP64 && precision != LBM_FP32))
        return LBM_EINVAL;
    if (lattice == LBM_D2Q9 && nz != 1) return LBM_EINVAL;
    const int64_t N = nx * ny * nz;
    const int64_t elem = precision == LBM_FP64 ? 8 : 4;
    if (N >= (1LL << 31) || N * elem >= (1LL << 32)) return LBM_EINVAL;
    lbe::Grid g;
    g.nx = (uint32_t)nx;
    g.ny = (uint32_t)ny;
    g.nz = (uint32_t)nz;
    g.N = (uint32_t)N;
    g.S = (uint32_t)N;
    g.nblocks = (uint32_t)((N + lbe::BX - 1) / lbe::BX);
    g.bpr = 0u;
    hipStream_t s;
    hipEvent_t e0, e1;
    if (hipStreamCreate(&s) != hipSuccess) return LBM_EDEVICE;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return LBM_EDEVICE;
    }
    auto launch = [&]() {
        auto go = [&](auto lat) {
            using L = decltype(lat);
            auto typed = [&](auto zero) {
                using T = decltype(zero);
                if (src2)
                    hipLaunchKernelGGL((lbe::k_adjoint_pattern<L, T>), dim3(g.nblocks),
                                       dim3(lbe::BX), 0, s, (const T*)src, (const T*)src2,
                                       (T*)dst, g);
                else
                    hipLaunchKernelGGL((lbe::k_pull_pattern<L, T>), dim3(g.nblocks),
                                       dim3(lbe::BX), 0, s, (const T*)src, (T*)dst, g);
            };
            if (precision == LBM_FP64) typed(0.0);
            else typed(0.0f);
        };
        if (lattice == LBM_D2Q9) go(lbe::D2Q9{});
        else if (lattice == LBM_D3Q15) go(lbe::D3Q15{});
        else go(lbe::D3Q19{});
    };
    launch();   // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(e1, s);
    int rc = LBM_OK;
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) rc = LBM_EDEVICE;
    float ms = 0.f;
    if (rc == LBM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = LBM_EDEVICE;
    if (ms_per_copy) *ms_per_copy = ms / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return rc;
}

}  // namespace

extern "C" int lbm_pull_pattern_copy(int lattice, int precision, void* dst, const void* src,
                                     int64_t nx, int64_t ny, int64_t nz, int32_t reps,
                                     double* ms_per_copy) {
    return pattern_copy(lattice, precision, dst, src, nullptr, nx, ny, nz, reps, ms_per_copy);
}

extern "C" int lbm_adjoint_pattern_copy(int lattice, int precision, void* dst, const void* f_src,
                                        const void* lam_src, int64_t nx, int64_t ny, int64_t nz,
                                        int32_t reps, double* ms_per_copy) {
    if (!lam_src) return LBM_EINVAL;
    return pattern_copy(lattice, precision, dst, f_src, lam_src, nx, ny, nz, reps, ms_per_copy);
}

extern "C" int lbm_aa_pattern_copy(int lattice, int precision, void* buf, int64_t nx, int64_t ny,
                                   int64_t nz, int32_t reps, double* ms_even, double* ms_odd) {
    if (!buf || nx < 1 || ny < 1 || nz < 1 || reps < 1) return LBM_EINVAL;
    if (lattice < 0 || lattice > 2 || (precision != LBM_FP64 && precision != LBM_FP32))
        return LBM_EINVAL;
    if (lattice == LBM_D2Q9 && nz != 1) return LBM_EINVAL;
    const int64_t N = nx * ny * nz;
    const int64_t elem = precision == LBM_FP64 ? 8 : 4;
    if (N >= (1LL << 31) || N * elem >= (1LL << 32)) return LBM_EINVAL;
    lbe::Grid g;
    g.nx = (uint32_t)nx;
    g.ny = (uint32_t)ny;
    g.nz = (uint32_t)nz;
    g.N = (uint32_t)N;
    g.S = (uint32_t)N;
    g.nblocks = (uint32_t)((N + lbe::BX - 1) / lbe::BX);
    g.bpr = 0u;
    hipStream_t s;
    hipEvent_t ev[3];
    if (hipStreamCreate(&s) != hipSuccess) return LBM_EDEVICE;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipStreamDestroy(s);
            return LBM_EDEVICE;
        }
    auto launch = [&](bool odd) {
        auto go = [&](auto lat) {
            using L = decltype(lat);
            auto typed = [&](auto zero) {
                using T = decltype(zero);
                if (odd)
                    hipLaunchKernelGGL((lbe::k_aa_pattern<L, T, true>), dim3(g.nblocks),
                                       dim3(lbe::BX), 0, s, (T*)buf, g);
                else
                    hipLaunchKernelGGL((lbe::k_aa_pattern<L, T, false>), dim3(g.nblocks),
                                       dim3(lbe::BX), 0, s, (T*)buf, g);
            };
            if (precision == LBM_FP64) typed(0.0);
            else typed(0.0f);
        };
        if (lattice == LBM_D2Q9) go(lbe::D2Q9{});
        else if (lattice == LBM_D3Q15) go(lbe::D3Q15{});
        else go(lbe::D3Q19{});
    };
    launch(false);   // warm-up pair
    launch(true);
    double t_even = 0.0, t_odd = 0.0;
    int rc = LBM_OK;
    for (int r = 0; r < reps && rc == LBM_OK; ++r) {
        (void)hipEventRecord(ev[0], s);
        launch(false);
        (void)hipEventRecord(ev[1], s);
        launch(true);
        (void)hipEventRecord(ev[2], s);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(ev[2]) != hipSuccess) {
            rc = LBM_EDEVICE;
            break;
        }
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, ev[0], ev[1]) != hipSuccess ||
            hipEventElapsedTime(&b, ev[1], ev[2]) != hipSuccess)
            rc = LBM_EDEVICE;
        t_even += a;
        t_odd += b;
    }
    if (ms_even) *ms_even = t_even / reps;
    if (ms_odd) *ms_odd = t_odd / reps;
    for (auto& e : ev) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(s);
    return rc;
}

extern "C" int lbm_blocked_pull_pattern_copy(int lattice, int precision, int32_t block,
                                             void* dst, const void* src, int64_t nx, int64_t ny,
                                             int64_t nz, int32_t reps, double* ms_per_copy) {
    if (!dst || !src || nx < 1 || ny < 1 || nz < 1 || reps < 1) return LBM_EINVAL;
    if (lattice < 0 || lattice > 2 || (precision != LBM_FP64 && precision != LBM_FP32))
        return LBM_EINVAL;
    if (lattice == LBM_D2Q9 && nz != 1) return LBM_EINVAL;
    if (block < 64 || block > (1 << 30) || (block & (block - 1))) return LBM_EINVAL;
    const int64_t N = nx * ny * nz;
    const int Q = lattice == LBM_D2Q9 ? 9 : (lattice == LBM_D3Q15 ? 15 : 19);
    const int64_t elem = precision == LBM_FP64 ? 8 : 4;
    if (N % block != 0 || N >= (1LL << 31) || N * Q * elem >= (1LL << 32)) return LBM_EINVAL;
    uint32_t lb = 0;
    while ((1 << lb) < block) ++lb;
    lbe::Grid g;
    g.nx = (uint32_t)nx;
    g.ny = (uint32_t)ny;
    g.nz = (uint32_t)nz;
    g.N = (uint32_t)N;
    g.S = (uint32_t)N;
    g.nblocks = (uint32_t)((N + lbe::BX - 1) / lbe::BX);
    g.bpr = 0u;
    hipStream_t s;
    hipEvent_t e0, e1;
    if (hipStreamCreate(&s) != hipSuccess) return LBM_EDEVICE;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return LBM_EDEVICE;
    }
    auto launch = [&]() {
        auto go = [&](auto lat) {
            using L = decltype(lat);
            auto typed = [&](auto zero) {
                using T = decltype(zero);
                hipLaunchKernelGGL((lbe::k_blocked_pull_pattern<L, T>), dim3(g.nblocks),
                                   dim3(lbe::BX), 0, s, (const T*)src, (T*)dst, g, lb);
            };
            if (precision == LBM_FP64) typed(0.0);
            else typed(0.0f);
        };
        if (lattice == LBM_D2Q9) go(lbe::D2Q9{});
        else if (lattice == LBM_D3Q15) go(lbe::D3Q15{});
        else go(lbe::D3Q19{});
    };
    launch();   // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) launch();
    (void)hipEventRecord(e1, s);
    int rc = LBM_OK;
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) rc = LBM_EDEVICE;
    float ms = 0.f;
    if (rc == LBM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = LBM_EDEVICE;
    if (ms_per_copy) *ms_per_copy = ms / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return rc;
}
