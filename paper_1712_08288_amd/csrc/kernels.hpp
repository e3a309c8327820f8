// Device code shared by the forward and adjoint kernels: the grid mapping,
// the pull addressing and the MRT collision.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lattice.hpp"

namespace lbe {

constexpr int BX = 256;            // threads per block, one node per thread

enum XBC : int { XBC_PERIODIC = 0, XBC_PRESSURE = 1, XBC_OUTFLOW = 2 };

// A node launch covers the node indices n = x + nx (y + ny z) in order, BX
// per block (64 per wave), whatever the row length: no lane idles except at
// the very end.  The hardware deals blocks to the eight XCDs round-robin
// (a remapping that gave each XCD one contiguous slab measured 8% slower).
struct Grid {
    uint32_t nx, ny, nz;
    uint32_t N;          // nx*ny*nz
    uint32_t S;          // N rounded up to whole population blocks (velocity-plane stride)
    uint32_t nblocks;    // blocks = ceil(N / BX)
    uint32_t bpr;        // nx / BX when BX divides nx (blocks per row), else 0
};

struct NodePos {
    uint32_t ix, iy, iz, n;
    bool in;
};

// ROWS (only when BX divides nx): every block lies in one row, so the row,
// y and z are block-uniform and stay in scalar registers.
template <bool ROWS = false>
__device__ __forceinline__ NodePos node_of_thread(const Grid& g) {
    const uint32_t b = blockIdx.x;
    NodePos p;
    p.n = b * BX + threadIdx.x;
    p.in = (b < g.nblocks) && (p.n < g.N);
    if constexpr (ROWS) {
        const uint32_t row = b / g.bpr;
        p.ix = (b - row * g.bpr) * BX + threadIdx.x;
        p.iz = row / g.ny;
        p.iy = row - p.iz * g.ny;
    } else {
        const uint32_t row = p.n / g.nx;
        p.ix = p.n - row * g.nx;
        p.iz = row / g.ny;
        p.iy = row - p.iz * g.ny;
    }
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
    T G[3];           // 3 rho0 g: the forcing term is F_i = w_i e_i.G
    T drho;           // pressure-jump boundary: the seam term is w_i drho
    T force[L::Q];    // the same two terms tabulated per population
    T seam[L::Q];
    T rho0, inv_rho0;
    double c0;        // 1 - b of Eq. (213)
    double rho0_d;
    double wall_scale;  // factor on the wall terms at this step (decaying data)
    const double* c1d;  // Eq. (211): per-link c1 added at the pull, or null
};

// Signed accumulate with a compile-time integer coefficient.
template <int C, class T>
__device__ __forceinline__ void macc(T& acc, T v) {
    if constexpr (C == 1) acc += v;
    else if constexpr (C == -1) acc -= v;
    else if constexpr (C != 0) acc = fma(T(C), v, acc);
}

// Forcing term F_i = 3 w_i rho0 e_i.g of population I, and the seam term
// w_i drho: from the tables (FTAB) or from the few runtime scalars they depend
// on.  A kernel loads only the arguments it uses into scalar registers; the
// scalars keep the adjoint and the FP64 step free of scalar-register spills,
// the tables keep the FP32 step's arithmetic lowest (both measured).
template <class L, int I, bool FTAB, class T>
__device__ __forceinline__ T force_of(const Params<L, T>& p) {
    if constexpr (FTAB) {
        return p.force[I];
    } else {
        T eg = T(0);
        macc<L::E[I][0]>(eg, p.G[0]);
        macc<L::E[I][1]>(eg, p.G[1]);
        macc<L::E[I][2]>(eg, p.G[2]);
        return T(L::W[I]) * eg;
    }
}
template <class L, int I, bool FTAB, class T>
__device__ __forceinline__ T seam_of(const Params<L, T>& p) {
    if constexpr (FTAB) return p.seam[I];
    else return T(L::W[I]) * p.drho;
}

// the step kernel's choice of the two forms above
template <class T>
inline constexpr bool kStepTables = std::is_same<T, float>::value;

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

// ---- the MRT transform in even/odd pair form (see Derived<L>) -------------
template <class L>
constexpr int NPAIR = (L::Q - 1) / 2;

template <class L, class T>
__device__ __forceinline__ void pair_split(const T (&x)[L::Q], T (&sp)[NPAIR<L>],
                                           T (&dp)[NPAIR<L>]) {
    unroll<NPAIR<L>>([&](auto P) {
        constexpr int pp = decltype(P)::value;
        constexpr int i = DER<L>.pi[pp];
        constexpr int ib = TAB<L>.opp[i];
        sp[pp] = x[i] + x[ib];
        dp[pp] = x[i] - x[ib];
    });
}

// (M x)_k for the non-conserved rows from the pair form of x
template <class L, class T>
__device__ __forceinline__ void moments_of(T x0, const T (&sp)[NPAIR<L>],
                                           const T (&dp)[NPAIR<L>], T (&m)[L::Q]) {
    unroll<L::Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        T acc = 0;
        if constexpr (!L::conserved(k)) {
            if constexpr (DER<L>.even[k]) {
                macc<TAB<L>.M[k][0]>(acc, x0);
                unroll<NPAIR<L>>([&](auto P) {
                    constexpr int pp = decltype(P)::value;
                    macc<TAB<L>.M[k][DER<L>.pi[pp]]>(acc, sp[pp]);
                });
            } else {
                unroll<NPAIR<L>>([&](auto P) {
                    constexpr int pp = decltype(P)::value;
                    macc<TAB<L>.M[k][DER<L>.pi[pp]]>(acc, dp[pp]);
                });
            }
        }
        m[k] = acc;
    });
}

// density deviation and momentum sum_i e_i x_i from the pair form
template <class L, class T>
__device__ __forceinline__ void conserved_of(T x0, const T (&sp)[NPAIR<L>],
                                             const T (&dp)[NPAIR<L>], T& rho, T (&j)[3]) {
    rho = x0;
    j[0] = j[1] = j[2] = 0;
    unroll<NPAIR<L>>([&](auto P) {
        constexpr int pp = decltype(P)::value;
        constexpr int i = DER<L>.pi[pp];
        rho += sp[pp];
        macc<L::E[i][0]>(j[0], dp[pp]);
        macc<L::E[i][1]>(j[1], dp[pp]);
        macc<L::E[i][2]>(j[2], dp[pp]);
    });
}

// m_k -= m^eq_k(drho, j) for the non-conserved rows (projection of Eq. (42))
template <class L, class T>
__device__ __forceinline__ void subtract_equilibrium(T (&m)[L::Q], T rho, const T (&j)[3],
                                                     T inv_rho0) {
    const T u[3] = {j[0] * inv_rho0, j[1] * inv_rho0, j[2] * inv_rho0};
    const T jj[6] = {j[0] * u[0], j[1] * u[1], j[2] * u[2],
                     j[0] * u[1], j[1] * u[2], j[0] * u[2]};
    unroll<L::Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (!L::conserved(k)) {
            if constexpr (DER<L>.A[k] != 0.0) m[k] -= T(DER<L>.A[k]) * rho;
            unroll<3>([&](auto X) {
                constexpr int x = decltype(X)::value;
                if constexpr (DER<L>.B[k][x] != 0.0) m[k] -= T(DER<L>.B[k][x]) * j[x];
            });
            unroll<6>([&](auto C) {
                constexpr int c = decltype(C)::value;
                if constexpr (DER<L>.C[k][c] != 0.0) m[k] -= T(DER<L>.C[k][c]) * jj[c];
            });
        }
    });
}

// y = M^T r over the non-conserved rows, in pair form:
// y_0 = e0, y_i = ev_p + od_p, y_ibar = ev_p - od_p
template <class L, class T>
__device__ __forceinline__ void back_transform(const T (&r)[L::Q], T& e0,
                                               T (&ev)[NPAIR<L>], T (&od)[NPAIR<L>]) {
    e0 = 0;
    unroll<L::Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (!L::conserved(k) && DER<L>.even[k]) macc<TAB<L>.M[k][0]>(e0, r[k]);
    });
    unroll<NPAIR<L>>([&](auto P) {
        constexpr int pp = decltype(P)::value;
        constexpr int i = DER<L>.pi[pp];
        T a = 0, b = 0;
        unroll<L::Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            if constexpr (!L::conserved(k)) {
                if constexpr (DER<L>.even[k]) macc<TAB<L>.M[k][i]>(a, r[k]);
                else macc<TAB<L>.M[k][i]>(b, r[k]);
            }
        });
        ev[pp] = a;
        od[pp] = b;
    });
}

// MRT collision of the Appendix plus forcing, in place:
// f <- f - M^{-1} S (M f - m^eq) + F with M^{-1} = M^T diag(1/|M_k|^2)
// (the rates arrive already divided by |M_k|^2).  m^eq is the projection of
// Eq. (42), so M f - m^eq = M (f - f^eq) exactly in real arithmetic.
// Optionally returns the non-equilibrium moments (M (f - f^eq))_k.
template <class L, class T, bool KEEP_NEQ = false, bool FTAB = false>
__device__ __forceinline__ void collide(T (&f)[L::Q], const Params<L, T>& p,
                                        Macro<L, T>& mac, T* neq = nullptr) {
    constexpr int NP = NPAIR<L>;
    T sp[NP], dp[NP];
    pair_split<L, T>(f, sp, dp);
    T rho, j[3];
    conserved_of<L, T>(f[0], sp, dp, rho, j);
    mac.rho = rho;
    mac.u[0] = j[0] * p.inv_rho0;
    mac.u[1] = j[1] * p.inv_rho0;
    mac.u[2] = j[2] * p.inv_rho0;
    T r[L::Q];
    moments_of<L, T>(f[0], sp, dp, r);
    subtract_equilibrium<L, T>(r, rho, j, p.inv_rho0);
    unroll<L::Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (KEEP_NEQ) neq[k] = r[k];
        r[k] *= p.rate[k];
    });
    T e0, ev[NP], od[NP];
    back_transform<L, T>(r, e0, ev, od);
    f[0] -= e0;
    unroll<NP>([&](auto P) {
        constexpr int pp = decltype(P)::value;
        constexpr int i = DER<L>.pi[pp];
        constexpr int ib = TAB<L>.opp[i];
        const T o = od[pp] - force_of<L, i, FTAB>(p);    // F_ibar = -F_i
        f[i] = f[i] - ev[pp] - o;
        f[ib] = f[ib] - ev[pp] + o;
    });
}

// Loads and stores through a uniform plane pointer and a 32-bit byte
// offset, so the address is a scalar base plus one VGPR (the caller keeps
// every plane below 4 GiB).
template <class T>
__device__ __forceinline__ T ld(const T* __restrict__ plane, uint32_t idx) {
    return *(const T*)((const char*)plane + idx * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st_nt(T* __restrict__ plane, uint32_t idx, T v) {
    __builtin_nontemporal_store(v, (T*)((char*)plane + idx * (uint32_t)sizeof(T)));
}

// Every array of Q populations per node (distributions, adjoint) is stored
// in blocks of NB consecutive nodes, each holding its Q planes of NB values
// one after the other: population i of node n lies at
// (n / NB) * Q * NB + i * NB + n % NB.  On the 256^3 pull pattern this moves
// 6.05 TB/s against 5.70 for whole planes of N values (blocks of 512 to
// 65536 nodes measured; from 2048 up FP32 is flat, FP64 best at 2048-4096).
constexpr uint32_t NB = 2048;

template <int Q>
__device__ __forceinline__ size_t pop_at(int i, uint32_t n) {
    return (size_t)(n / NB) * ((size_t)NB * Q) + (size_t)i * NB + (n % NB);
}
template <int Q, class T>
__device__ __forceinline__ T ldp(const T* __restrict__ a, int i, uint32_t n) {
    return a[pop_at<Q>(i, n)];
}
template <int Q, class T>
__device__ __forceinline__ void stp_nt(T* __restrict__ a, int i, uint32_t n, T v) {
    __builtin_nontemporal_store(v, a + pop_at<Q>(i, n));
}

// ----------------------------------------------------------------------------
// link lookup: the links of a node are contiguous, sorted by direction.
struct NodeLinks {
    uint32_t mask;   // bit i set if direction i is a cut link
    uint32_t base;   // index of the node's first link
};

// Per-node and per-wave metadata of the geometry.  Links are sorted by node,
// then direction, so the links of one 64-node wave of a node launch are
// contiguous: a node's first link is its wave's first link plus the count of
// links at the wave's earlier nodes, kept in bits 19..30 of the info word
// (at most 64 * (Q - 1) = 1152 links per wave).
struct NodeMeta {
    const uint32_t* __restrict__ info;   // bit 31: solid; bits 19..30: link offset
                                         // within the wave; bits 0..Q-1: cut-link directions
    const uint2* __restrict__ wave;      // per wave: x = kind (bits 0..1: 0 mixed,
                                         // 1 all fluid without links, 2 no fluid), link
                                         // count (bits 2..15) and the eighths of 8
                                         // lanes without a fluid node (bits 16..23);
                                         // y = first link
};

enum WaveKind : uint32_t { WAVE_MIXED = 0, WAVE_PLAIN = 1, WAVE_IDLE = 2 };

constexpr uint32_t kInfoSolid = 0x80000000u;
constexpr uint32_t kInfoMask = (1u << 19) - 1u;
constexpr int kInfoOffsetShift = 19;
constexpr uint32_t kInfoOffsetMax = 0xFFFu;

__device__ __forceinline__ bool is_solid(uint32_t info) { return (info >> 31) != 0; }
__device__ __forceinline__ uint32_t wave_kind(uint2 w) { return w.x & 3u; }
__device__ __forceinline__ uint32_t wave_links(uint2 w) { return (w.x >> 2) & 0x3FFFu; }
// A mixed wave's lanes in a 64-byte segment of a plane without fluid nodes
// (16 lanes in FP32, 8 in FP64) neither read nor write it.  Smaller segments
// are still written whole (NaN at solid lanes): partial writes cost HBM
// read-modify-write cycles.
template <class T>
__device__ __forceinline__ bool lane_in_live_segment(uint32_t wave_x, uint32_t lane) {
    if constexpr (sizeof(T) == 4)
        return ((wave_x >> (16u + 2u * (lane >> 4))) & 3u) != 3u;
    else
        return ((wave_x >> (16u + (lane >> 3))) & 1u) == 0u;
}

// the wave of a node launch that holds node n
__device__ __forceinline__ uint32_t wave_of_node(const Grid&, uint32_t n) { return n / 64; }

// links of a node whose wave's first link index is known
__device__ __forceinline__ NodeLinks node_links(uint32_t info, uint32_t wave_base) {
    NodeLinks r;
    r.mask = info & kInfoMask;
    r.base = wave_base + ((info >> kInfoOffsetShift) & kInfoOffsetMax);
    return r;
}

__device__ __forceinline__ NodeLinks node_links(const NodeMeta& nm, const Grid& g,
                                                uint32_t info, uint32_t n) {
    if (!(info & kInfoMask)) return NodeLinks{0u, 0u};
    return node_links(info, nm.wave[wave_of_node(g, n)].y);
}

__device__ __forceinline__ uint32_t link_index(const NodeLinks& nl, int i) {
    return nl.base + __popc(nl.mask & ((1u << i) - 1u));
}

// Read the planes of a pull: f_i = A_i(x - e_i) (+ seam term).  With PRED
// the planes of cut-link directions are not read.
template <class L, class T, int XB, bool PRED = false, bool FTAB = false>
__device__ __forceinline__ void pull_planes(const T* __restrict__ A, const Grid& g,
                                            const NodePos& pos, const Params<L, T>& p,
                                            const NodeLinks& nl, T (&f)[L::Q]) {
    const Pull<XB> pl(g, pos);
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (PRED && i > 0 && ((nl.mask >> i) & 1u)) {
            f[i] = 0;
            return;
        }
        f[i] = ldp<L::Q>(A, i, pl.template src<L, i>());
        if constexpr (XB == XBC_PRESSURE && L::E[i][0] != 0) {
            const int sg = seam_sign<L, i>(pos.ix, g.nx);
            if (sg > 0) f[i] += seam_of<L, i, FTAB>(p);
            else if (sg < 0) f[i] -= seam_of<L, i, FTAB>(p);
        }
    });
}

// Eq. (211): a cut-link slot holds the terms at t only; the pull completes it
// with c1 f_ibar(x, t), the value just advected from x + e_i.  c1d is indexed
// like nl.base.
template <class L, class T>
__device__ __forceinline__ void complete_two_node(const double* __restrict__ c1d,
                                                  const NodeLinks& nl, T (&f)[L::Q]) {
    if (!nl.mask) return;
    uint32_t kk = nl.base;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ib = TAB<L>.opp[i];
        if constexpr (i > 0) {
            const uint32_t bit = (nl.mask >> i) & 1u;
            if (bit) {
                const double c = c1d[kk];
                if (c != 0.0) f[i] = (T)((double)f[i] + c * (double)f[ib]);
            }
            kk += bit;
        }
    });
}

// Cut-link directions take their link slot (links are sorted by direction,
// so a running index replaces a popcount).
template <class L, class T>
__device__ __forceinline__ void apply_links(const T* __restrict__ wa, const Params<L, T>& p,
                                            const NodeLinks& nl, T (&f)[L::Q]) {
    if (!nl.mask) return;
    uint32_t k = nl.base;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (i > 0) {
            const uint32_t bit = (nl.mask >> i) & 1u;
            if (bit) f[i] = wa[k];
            k += bit;
        }
    });
    if (p.c1d) complete_two_node<L, T>(p.c1d, nl, f);
}

// Per-wave cooperative handling of cut links.  The links of one wave of a
// node launch are contiguous (sorted by node, then direction); lane l carries
// the wave's link l of the first 64, and values move between that lane and
// the lane of the link's fluid node through a per-wave LDS slab.
template <class T>
struct LinkStage {
    T v[4][64];
};

// order the wave's LDS writes before the other lanes' reads (the LDS executes
// one wave's instructions in order; this keeps the compiler from moving them)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pulled values of cut-link directions: f_i(x_f, t) = wa[k].  nl.base is the
// node's first link relative to the wave's first link wbase; wa0 =
// wa[wbase + lane] for lanes below the wave's link count (else 0), read in
// advance by every lane.
template <class L, class T>
__device__ __forceinline__ void wave_link_values(const T* __restrict__ wa, uint32_t wbase,
                                                 uint32_t lane, T wa0, const NodeLinks& nl,
                                                 LinkStage<T>& st, T (&f)[L::Q]) {
    st.v[0][lane] = wa0;
    wave_lds_sync();
    if (nl.mask) {
        uint32_t k = nl.base;
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (i > 0) {
                const uint32_t bit = (nl.mask >> i) & 1u;
                if (bit) f[i] = k < 64u ? st.v[0][k] : wa[wbase + k];
                k += bit;
            }
        });
    }
    wave_lds_sync();
}

// Eq. (211) completion for a mixed wave (see complete_two_node; c1d indexed
// like nl.base): the c1 values of the wave's first 64 links come from their
// link lanes, which load them coalesced with the slot reads (c1v =
// c1d[lane] below the wave's link count), through a per-wave LDS row.
template <class L, class T>
__device__ __forceinline__ void wave_two_node(const double* __restrict__ c1d, uint32_t lane,
                                              double c1v, const NodeLinks& nl,
                                              double (&c1s)[64], T (&f)[L::Q]) {
    c1s[lane] = c1v;
    wave_lds_sync();
    if (!nl.mask) return;
    uint32_t k = nl.base;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int ib = TAB<L>.opp[i];
        if constexpr (i > 0) {
            const uint32_t bit = (nl.mask >> i) & 1u;
            if (bit) {
                const double c = k < 64u ? c1s[k] : c1d[k];
                if (c != 0.0) f[i] = (T)((double)f[i] + c * (double)f[ib]);
            }
            k += bit;
        }
    });
}

// Pull the pre-collision state f(x, t) of one fluid node.
template <class L, class T, int XB, bool PRED = false, bool FTAB = false>
__device__ __forceinline__ void pull(const T* __restrict__ A, const T* __restrict__ wa,
                                     const Grid& g, const NodePos& pos,
                                     const Params<L, T>& p, const NodeLinks& nl,
                                     T (&f)[L::Q]) {
    pull_planes<L, T, XB, PRED, FTAB>(A, g, pos, p, nl, f);
    apply_links<L, T>(wa, p, nl, f);
}

// The value f_i(n, t) that a pull of direction i at fluid node n would read
// from A (no link override); used by link kernels.
template <class L, class T, int XB>
__device__ __forceinline__ T pull_one(const T* __restrict__ A, const Grid& g,
                                      const Params<L, T>& p, uint32_t n, int i) {
    const uint32_t ix = n % g.nx, r = n / g.nx;
    const uint32_t iy = r % g.ny, iz = r / g.ny;
    T out = 0;
    unroll<L::Q>([&](auto I) {
        constexpr int ii = decltype(I)::value;
        if (ii == i) {
            int sx = (int)ix - L::E[ii][0];
            int sg = 0;
            if (XB == XBC_OUTFLOW) {
                sx = sx < 0 ? 0 : (sx >= (int)g.nx ? (int)g.nx - 1 : sx);
            } else {
                if (sx < 0) { sx += g.nx; sg = 1; }
                else if (sx >= (int)g.nx) { sx -= g.nx; sg = -1; }
            }
            int sy = (int)iy - L::E[ii][1];
            sy = sy < 0 ? sy + (int)g.ny : (sy >= (int)g.ny ? sy - (int)g.ny : sy);
            int sz = (int)iz - L::E[ii][2];
            sz = sz < 0 ? sz + (int)g.nz : (sz >= (int)g.nz ? sz - (int)g.nz : sz);
            const uint32_t src = (uint32_t)sx + g.nx * ((uint32_t)sy + g.ny * (uint32_t)sz);
            out = ldp<L::Q>(A, ii, src);
            if (XB == XBC_PRESSURE) {
                if (sg > 0) out += seam_of<L, ii, false>(p);
                else if (sg < 0) out -= seam_of<L, ii, false>(p);
            }
        }
    });
    return out;
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
