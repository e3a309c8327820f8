// Device code shared by the forward and adjoint kernels: the grid mapping,
// the pull addressing and the MRT collision.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattice.hpp"

namespace lbe {

constexpr int BX = 256;            // threads per block, one node per thread
constexpr int NXCD = 8;            // compute dies on MI355X (blocks go round-robin)

enum XBC : int { XBC_PERIODIC = 0, XBC_PRESSURE = 1, XBC_OUTFLOW = 2 };

// A launch covers rows of nx nodes in chunks of BX threads.  Blocks are
// dealt to the eight XCDs round-robin by hardware; `remap` turns the block
// id into a logical id so that each XCD sweeps one contiguous slab of rows
// and the y/z-neighbour rows a pull touches stay in that XCD's L2.
struct Grid {
    uint32_t nx, ny, nz;
    uint32_t N;          // nx*ny*nz
    uint32_t bpr;        // blocks per row
    uint32_t nblocks;    // logical blocks = bpr*ny*nz
    uint32_t chunk;      // ceil(nblocks / NXCD) when remapping, else 0
};

struct NodePos {
    uint32_t ix, iy, iz, n;
    bool in;
};

__device__ __forceinline__ NodePos node_of_thread(const Grid& g) {
    uint32_t b = blockIdx.x;
    if (g.chunk) b = (b % NXCD) * g.chunk + b / NXCD;
    NodePos p;
    const uint32_t row = b / g.bpr;
    const uint32_t xb = b - row * g.bpr;
    p.ix = xb * BX + threadIdx.x;
    p.iy = row % g.ny;
    p.iz = row / g.ny;
    p.in = (b < g.nblocks) && (p.ix < g.nx);
    p.n = p.ix + g.nx * (p.iy + g.ny * p.iz);
    return p;
}

// Node indices of the nine (y, z) neighbour rows and three x neighbours of
// a node; element [e + 1] is the coordinate x - e (the pull source of a
// population moving with e).
template <int XB>
struct Pull {
    uint32_t xs[3];
    uint32_t row[3][3];

    __device__ __forceinline__ Pull(const Grid& g, const NodePos& p) {
        const uint32_t xm = p.ix == 0 ? g.nx - 1 : p.ix - 1;
        uint32_t xp = p.ix + 1 == g.nx ? 0u : p.ix + 1;
        if (XB == XBC_OUTFLOW && p.ix + 1 == g.nx) xp = p.ix;
        xs[0] = xp;       // e_x = -1 reads x + 1
        xs[1] = p.ix;
        xs[2] = xm;       // e_x = +1 reads x - 1
        const uint32_t ys[3] = {p.iy + 1 == g.ny ? 0u : p.iy + 1, p.iy,
                                p.iy == 0 ? g.ny - 1 : p.iy - 1};
        const uint32_t zs[3] = {p.iz + 1 == g.nz ? 0u : p.iz + 1, p.iz,
                                p.iz == 0 ? g.nz - 1 : p.iz - 1};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) row[a][c] = g.nx * (ys[a] + g.ny * zs[c]);
    }

    template <class L, int I>
    __device__ __forceinline__ uint32_t src() const {
        return xs[L::E[I][0] + 1] + row[L::E[I][1] + 1][L::E[I][2] + 1];
    }
};

// Seam sign of the pressure-jump x boundary for population I at x = ix:
// +1 when it crossed from x = nx-1 to 0, -1 for the opposite crossing.
template <class L, int I>
__device__ __forceinline__ int seam_sign(uint32_t ix, uint32_t nx) {
    if constexpr (L::E[I][0] == 1) return ix == 0 ? 1 : 0;
    else if constexpr (L::E[I][0] == -1) return ix + 1 == nx ? -1 : 0;
    else return 0;
}

template <class L, class T>
struct Params {
    T rate[L::Q];     // s_k / |M_k|^2, zero for conserved rows
    T force[L::Q];    // 3 w_i rho0 e_i.g
    T seam[L::Q];     // w_i drho (pressure-jump boundary)
    T rho0, inv_rho0;
    double c0;        // 1 - b of Eq. (213)
    double rho0_d;
};

// Signed accumulate with a compile-time integer coefficient.
template <int C, class T>
__device__ __forceinline__ void macc(T& acc, T v) {
    if constexpr (C == 1) acc += v;
    else if constexpr (C == -1) acc -= v;
    else if constexpr (C != 0) acc = fma(T(C), v, acc);
}

template <class L, class T>
struct Macro {
    T rho;       // density deviation sum_i delta f_i
    T u[3];      // sum_i e_i f_i / rho0
};

template <class L, class T>
__device__ __forceinline__ Macro<L, T> moments(const T (&f)[L::Q], T inv_rho0) {
    Macro<L, T> m;
    T r = 0, j0 = 0, j1 = 0, j2 = 0;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        r += f[i];
        macc<L::E[i][0]>(j0, f[i]);
        macc<L::E[i][1]>(j1, f[i]);
        macc<L::E[i][2]>(j2, f[i]);
    });
    m.rho = r;
    m.u[0] = j0 * inv_rho0;
    m.u[1] = j1 * inv_rho0;
    m.u[2] = j2 * inv_rho0;
    return m;
}

// Equilibrium of Eq. (42) (c = 1, c_s^2 = 1/3) in deviation form:
// w_i [drho + rho0 (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)].
template <class L, class T, int I>
__device__ __forceinline__ T feq(const Macro<L, T>& m, T rho0) {
    T eu = 0;
    macc<L::E[I][0]>(eu, m.u[0]);
    macc<L::E[I][1]>(eu, m.u[1]);
    macc<L::E[I][2]>(eu, m.u[2]);
    const T uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
    const T poly = eu * (T(3) + T(4.5) * eu) - T(1.5) * uu;
    return T(L::W[I]) * (m.rho + rho0 * poly);
}

// MRT collision of the Appendix plus forcing, in place:
// f <- f - M^{-1} S M (f - f^eq) + F with M^{-1} = M^T diag(1/|M_k|^2).
template <class L, class T>
__device__ __forceinline__ void collide(T (&f)[L::Q], const Params<L, T>& p,
                                        Macro<L, T>& mac) {
    mac = moments<L, T>(f, p.inv_rho0);
    T d[L::Q];
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        d[i] = f[i] - feq<L, T, i>(mac, p.rho0);
    });
    T m[L::Q];
    unroll<L::Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (!L::conserved(k)) {
            T acc = 0;
            unroll<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                macc<TAB<L>.M[k][i]>(acc, d[i]);
            });
            m[k] = acc * p.rate[k];
        }
    });
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        T acc = 0;
        unroll<L::Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            if constexpr (!L::conserved(k)) macc<TAB<L>.M[k][i]>(acc, m[k]);
        });
        f[i] = f[i] - acc + p.force[i];
    });
}

// ----------------------------------------------------------------------------
// link lookup: the links of a node are contiguous, sorted by direction.
struct NodeLinks {
    uint32_t mask;   // bit i set if direction i is a cut link
    uint32_t base;   // index of the node's first link
};

__device__ __forceinline__ NodeLinks node_links(int32_t nw, const uint8_t* __restrict__ lkdir) {
    NodeLinks r{0u, 0u};
    if (nw > 0) {
        const uint32_t cnt = (uint32_t)nw >> 26;
        r.base = (uint32_t)nw & 0x3FFFFFFu;
        for (uint32_t k = 0; k < cnt; ++k) r.mask |= 1u << lkdir[r.base + k];
    }
    return r;
}

__device__ __forceinline__ uint32_t link_index(const NodeLinks& nl, int i) {
    return nl.base + __popc(nl.mask & ((1u << i) - 1u));
}

// Pull the pre-collision state f(x, t) of one fluid node.
template <class L, class T, int XB>
__device__ __forceinline__ void pull(const T* __restrict__ A, const T* __restrict__ wa,
                                     const Grid& g, const NodePos& pos,
                                     const Params<L, T>& p, const NodeLinks& nl,
                                     T (&f)[L::Q]) {
    const Pull<XB> pl(g, pos);
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        f[i] = A[(size_t)i * g.N + pl.template src<L, i>()];
        if constexpr (XB == XBC_PRESSURE && L::E[i][0] != 0) {
            const int sg = seam_sign<L, i>(pos.ix, g.nx);
            if (sg > 0) f[i] += p.seam[i];
            else if (sg < 0) f[i] -= p.seam[i];
        }
    });
    if (nl.mask) {
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0)
                if ((nl.mask >> i) & 1u) f[i] = wa[link_index(nl, i)];
        });
    }
}

// Block-wide sum of one double per thread (all threads must call).
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[BX / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) part[wid] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BX / 64; ++w) s += part[w];
    return s;   // valid in thread 0
}

}  // namespace lbe
