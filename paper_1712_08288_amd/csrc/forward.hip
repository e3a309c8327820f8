// Forward kernels: the fused pull collide-stream step with the single-node
// boundary scheme, initialisation, observation and reductions.
//
// Storage (per precision T = float or double, deviation form f - w rho0):
//   A            post-collision value f'_i(n, t-1) at every node n, in
//                blocks of NB nodes that each hold their Q direction runs
//                (element pop_at<Q>(i, n));
//   wa[k]        for cut link k = (x_f, i): the value f_i(x_f, t) produced by
//                Eq. (213) during the previous step (the "write-ahead" slot).
// Pulling f_i(x, t) = A_i(x - e_i) (+ seam term), or wa[k] on a cut link,
// gives the pre-collision state of Eq. (21) at time t.
#include <algorithm>
#include <mutex>

#include "engine.hpp"
#include "kernels.hpp"

namespace lbe {

static_assert(BX == kBlock && BX % 64 == 0, "node launches use kBlock-thread blocks");

// ----------------------------------------------------------------------------
// the step: pull, collide, store, and evaluate Eq. (213) for the node's links

// The links of one wave are contiguous (sorted by node, then direction), so
// the wave handles its first 64 cooperatively: lane l carries the wave's
// link l, and values move between that lane and the lane of the link's
// fluid node through a per-wave LDS slab.  Slot reads, coefficient reads and
// slot writes are then coalesced, and the slot reads need no per-node
// metadata, so they are issued with the plane reads.  Links past the 64th
// (rare: long wall rows) are read and written by their node's lane directly;
// straight-line code keeps the register count of the step at its minimum.

// Eq. (213) for every cut link of the wave, from the pre-collision (fpre)
// and post-collision (f) values at its fluid node, into the link slots of
// the next step; nlw links in the wave.  REC: also the link values of the
// step record (f_ibar(y, t), f'_i(y, t), f'_ibar(y, t)).
template <class L, class T, bool REC>
__device__ __forceinline__ void wave_link_tail(const NodeLinks& nl, const T (&fpre)[L::Q],
                                               const T (&f)[L::Q],
                                               const LinkCoefT<T>* __restrict__ lkcoef,
                                               T* __restrict__ waB, double c0d, double ws,
                                               uint32_t wbase,
                                               uint32_t nlw, uint32_t lane, LinkStage<T>& st,
                                               const StepRecord<T>& rec) {
    if (nl.mask) {
        uint32_t k = nl.base;
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int ib = TAB<L>.opp[i];
            if constexpr (i > 0) {
                const uint32_t bit = (nl.mask >> i) & 1u;
                if (bit) {
                    if (k < 64u) {
                        st.v[0][k] = fpre[i];
                        st.v[1][k] = fpre[ib];
                        st.v[2][k] = f[i];
                        st.v[3][k] = f[ib];
                    } else {
                        const LinkCoefT<T> c = lkcoef[wbase + k];
                        const double v = c0d * (double)fpre[i] + c.c1 * (double)fpre[ib] +
                                         c.c2 * (double)f[i] + c.c3 * (double)f[ib] + ws * c.wall;
                        waB[wbase + k] = (T)v;
                        if constexpr (REC) {
                            rec.fib[wbase + k] = fpre[ib];
                            rec.fpi[wbase + k] = f[i];
                            rec.fpib[wbase + k] = f[ib];
                        }
                    }
                }
                k += bit;
            }
        });
    }
    wave_lds_sync();
    if (lane < nlw) {
        const LinkCoefT<T> c = lkcoef[wbase + lane];
        const double v = c0d * (double)st.v[0][lane] + c.c1 * (double)st.v[1][lane] +
                         c.c2 * (double)st.v[2][lane] + c.c3 * (double)st.v[3][lane] + ws * c.wall;
        waB[wbase + lane] = (T)v;
        if constexpr (REC) {
            rec.fib[wbase + lane] = st.v[1][lane];
            rec.fpi[wbase + lane] = st.v[2][lane];
            rec.fpib[wbase + lane] = st.v[3][lane];
        }
    }
}

// The objective term of one fluid node (see StepObjective): u_x for the mean
// velocity, the plane weight times the density deviation for the pressure
// drop.
__device__ __forceinline__ double objective_term(const StepObjective& ob, uint32_t ix,
                                                 double drho, double ux) {
    if (ob.kind == 3)
        return ((ix == ob.x_in ? ob.a_in : 0.0) - (ix == ob.x_out ? ob.a_out : 0.0)) * drho;
    return ux;
}

// Waves are classified on the host (one scalar load per wave): a wave whose
// 64 nodes are all fluid and free of cut links issues its pulls at once and
// collides; a wave without fluid exits.  A mixed wave reads every plane as
// if its nodes were plain (solid and cut-link slots included) and replaces
// the cut-link directions from their slots.  Its solid lanes store NaN into
// their own slots, which nothing reads: a full store keeps every written
// cache line whole (partial lines cost HBM read-modify-write cycles).  Lanes
// whose 64-byte segment of the planes holds no fluid node skip both.
// REC: also write the step record (StepRecord) for the reverse sweep.
template <class L, class T, int XB, bool ROWS, bool REC>
__global__ void __launch_bounds__(BX)
k_step(const T* __restrict__ A, T* __restrict__ B, const T* __restrict__ waA,
       T* __restrict__ waB, NodeMeta nm, const LinkCoefT<T>* __restrict__ lkcoef,
       Grid g, Params<L, T> p, StepObjective ob, StepRecord<T> rec) {
    __shared__ LinkStage<T> stage[BX / 64];
    __shared__ double c1s[BX / 64][64];   // Eq. (211): c1 of the wave's links
    const NodePos pos = node_of_thread<ROWS>(g);
    const uint32_t lb = blockIdx.x;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint2 wv = lb < g.nblocks ? nm.wave[lb * (BX / 64) + wid] : uint2{WAVE_IDLE, 0u};
    const uint32_t kind = wave_kind(wv);
    double obj_local = 0.0;
    if (kind == WAVE_PLAIN) {
        T f[L::Q];
        pull<L, T, XB, false, kStepTables<T>>(A, waA, g, pos, p, NodeLinks{0u, 0u}, f);
        Macro<L, T> mac;
        collide<L, T, false, kStepTables<T>>(f, p, mac);
        if (ob.acc) obj_local = objective_term(ob, pos.ix, (double)mac.rho, (double)mac.u[0]);
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            stp_nt<L::Q>(B, i, pos.n, f[i]);
        });
        if constexpr (REC)
            for (int a = 0; a < L::D; ++a) st_nt(rec.u + (size_t)a * g.S, pos.n, mac.u[a]);
    } else if (kind == WAVE_MIXED) {
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t nlw = wave_links(wv), wbase = wv.y;
        // slot reads and the info word first, the plane reads without
        // waiting for either
        const T wa0 = lane < nlw ? waA[wbase + lane] : T(0);
        const double c1v = p.c1d && lane < nlw ? p.c1d[wbase + lane] : 0.0;
        const bool live = pos.in && lane_in_live_segment<T>(wv.x, lane);
        const uint32_t info = live ? nm.info[pos.n] : kInfoSolid;
        T f[L::Q];
        if (live) {
            pull_planes<L, T, XB, false, kStepTables<T>>(A, g, pos, p, NodeLinks{0u, 0u}, f);
        } else {
            unroll<L::Q>([&](auto I) { f[decltype(I)::value] = T(0); });
        }
        const bool sol = is_solid(info);
        const NodeLinks nl = sol ? NodeLinks{0u, 0u} : node_links(info, 0u);
        wave_link_values<L, T>(waA, wbase, lane, wa0, nl, stage[wid], f);
        if (p.c1d) wave_two_node<L, T>(p.c1d + wbase, lane, c1v, nl, c1s[wid], f);
        T fpre[L::Q];
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            fpre[i] = f[i];
        });
        Macro<L, T> mac;
        collide<L, T, false, kStepTables<T>>(f, p, mac);
        if (live) {
            if (!sol && ob.acc) obj_local = objective_term(ob, pos.ix, (double)mac.rho, (double)mac.u[0]);
            const T nan = (T)__builtin_nan("");
            unroll<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                stp_nt<L::Q>(B, i, pos.n, sol ? nan : f[i]);
            });
            if constexpr (REC)
                for (int a = 0; a < L::D; ++a)
                    st_nt(rec.u + (size_t)a * g.S, pos.n, sol ? nan : mac.u[a]);
        }
        wave_link_tail<L, T, REC>(nl, fpre, f, lkcoef, waB, p.c0, p.wall_scale, wbase, nlw,
                                  lane, stage[wid], rec);
    }
    if (ob.acc) {   // uniform over the launch
        const double s = block_sum(obj_local);
        if (threadIdx.x == 0 && lb < g.nblocks) ob.acc[lb] += ob.w * s;
    }
}

// ----------------------------------------------------------------------------
// initial state: scatter f(x, 0) into the slots the first pull reads
template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_init(const double* __restrict__ df, const double* __restrict__ rho,
       const double* __restrict__ u, T* __restrict__ A, T* __restrict__ wa,
       NodeMeta nm, Grid g, Params<L, T> p) {
    const NodePos pos = node_of_thread(g);
    if (!pos.in) return;
    const uint32_t info = nm.info[pos.n];
    if (is_solid(info)) return;
    const NodeLinks nl = node_links(nm, g, info, pos.n);
    double f[L::Q];
    if (df) {
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            f[i] = df[(size_t)i * g.N + pos.n];
        });
    } else {
        Macro<L, double> m;
        m.rho = (rho ? rho[pos.n] : p.rho0_d) - p.rho0_d;
        m.u[0] = m.u[1] = m.u[2] = 0.0;
        if (u)
            for (int a = 0; a < L::D; ++a) m.u[a] = u[(size_t)pos.n * L::D + a];
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            f[i] = feq<L, double, i>(m, p.rho0_d);
        });
    }
    const Pull<XB> pl(g, pos);
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (i > 0 && ((nl.mask >> i) & 1u)) {
            const uint32_t k = link_index(nl, i);
            // Eq. (211): the first pull adds c1 f_ibar(x_f, 0) to the slot
            const double c = p.c1d ? p.c1d[k] : 0.0;
            wa[k] = (T)(f[i] - c * f[TAB<L>.opp[i]]);
            return;
        }
        // the outlet column's -x populations share their slot with the pull
        // of node (nx-2, y, z); that node's value is kept unless it is solid
        if constexpr (XB == XBC_OUTFLOW && L::E[i][0] == -1)
            if (pos.ix + 1 == g.nx && !is_solid(nm.info[pos.n - 1])) return;
        T v = (T)f[i];
        if constexpr (XB == XBC_PRESSURE && L::E[i][0] != 0) {
            const int sg = seam_sign<L, i>(pos.ix, g.nx);
            if (sg > 0) v -= seam_of<L, i, false>(p);
            else if (sg < 0) v += seam_of<L, i, false>(p);
        }
        A[pop_at<L::Q>(i, pl.template src<L, i>())] = v;
    });
}

// ----------------------------------------------------------------------------
// observation: moments or the full distribution of f(x, t), NaN at solids
template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_observe(const T* __restrict__ A, const T* __restrict__ wa, NodeMeta nm,
          Grid g, Params<L, T> p, double* __restrict__ rho, double* __restrict__ u,
          double* __restrict__ df) {
    const NodePos pos = node_of_thread(g);
    if (!pos.in) return;
    const uint32_t info = nm.info[pos.n];
    const double nan = __builtin_nan("");
    if (is_solid(info)) {
        if (rho) rho[pos.n] = nan;
        if (u)
            for (int a = 0; a < L::D; ++a) u[(size_t)pos.n * L::D + a] = nan;
        if (df)
            for (int i = 0; i < L::Q; ++i) df[(size_t)i * g.N + pos.n] = nan;
        return;
    }
    const NodeLinks nl = node_links(nm, g, info, pos.n);
    T f[L::Q];
    pull<L, T, XB, true>(A, wa, g, pos, p, nl, f);
    if (df) {
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            df[(size_t)i * g.N + pos.n] = (double)f[i];
        });
    }
    if (rho || u) {
        double r = 0, j[3] = {0, 0, 0};
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double v = (double)f[i];
            r += v;
            macc<L::E[i][0]>(j[0], v);
            macc<L::E[i][1]>(j[1], v);
            macc<L::E[i][2]>(j[2], v);
        });
        if (rho) rho[pos.n] = p.rho0_d + r;
        if (u)
            for (int a = 0; a < L::D; ++a) u[(size_t)pos.n * L::D + a] = j[a] / p.rho0_d;
    }
}

// per-block sums of drho and sum e f (= rho0 u) over fluid nodes
template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_mass(const T* __restrict__ A, const T* __restrict__ wa, NodeMeta nm,
       Grid g, Params<L, T> p, double* __restrict__ partials) {
    const NodePos pos = node_of_thread(g);
    const uint32_t info = pos.in ? nm.info[pos.n] : kInfoSolid;
    double r = 0, j[3] = {0, 0, 0};
    if (!is_solid(info)) {
        const NodeLinks nl = node_links(nm, g, info, pos.n);
        T f[L::Q];
        pull<L, T, XB, true>(A, wa, g, pos, p, nl, f);
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double v = (double)f[i];
            r += v;
            macc<L::E[i][0]>(j[0], v);
            macc<L::E[i][1]>(j[1], v);
            macc<L::E[i][2]>(j[2], v);
        });
    }
    const uint32_t b = blockIdx.x;
    double vals[4] = {r, j[0], j[1], j[2]};
    for (int c = 0; c < 1 + L::D; ++c) {
        const double s = block_sum(vals[c]);
        if (threadIdx.x == 0 && b < g.nblocks) partials[(size_t)b * (1 + L::D) + c] = s;
    }
}

// per-block sums of a_p (rho - rho0) over the fluid nodes of the planes
// x = x_in and x = x_out: thread t covers node (x_p, r) of plane p = t / R,
// r = t % R, R = ny nz
template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_plane_density(const T* __restrict__ A, const T* __restrict__ wa, NodeMeta nm, Grid g,
                Params<L, T> p, uint32_t x_in, uint32_t x_out, double a_in, double a_out,
                double* __restrict__ partials) {
    const uint32_t R = g.ny * g.nz;
    const uint32_t t = blockIdx.x * BX + threadIdx.x;
    double v = 0.0;
    if (t < 2u * R) {
        const uint32_t plane = t / R, r = t - plane * R;
        NodePos pos;
        pos.ix = plane ? x_out : x_in;
        pos.iz = r / g.ny;
        pos.iy = r - pos.iz * g.ny;
        pos.n = pos.ix + g.nx * r;
        pos.in = true;
        const uint32_t info = nm.info[pos.n];
        if (!is_solid(info)) {
            const NodeLinks nl = node_links(nm, g, info, pos.n);
            T f[L::Q];
            pull<L, T, XB, true>(A, wa, g, pos, p, nl, f);
            double r0 = 0.0;
            unroll<L::Q>([&](auto I) { r0 += (double)f[decltype(I)::value]; });
            v = (plane ? -a_out : a_in) * r0;
        }
    }
    const double s = block_sum(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// momentum exchange of the last step on each link; `post` holds f'(t-1) at
// every node and the link slots of f_i(x_f, t)
template <class L, class T, int XB>
__device__ __forceinline__ double link_value(const T* __restrict__ B, const T* __restrict__ wa,
                                             const Grid& g, const Params<L, T>& p,
                                             uint32_t k, uint32_t n, int i) {
    double v = (double)wa[k];
    if (p.c1d) {
        const double c = p.c1d[k];
        if (c != 0.0) {
            int ib = 0;
            unroll<L::Q>([&](auto I) {
                constexpr int ii = decltype(I)::value;
                if (ii == i) ib = TAB<L>.opp[ii];
            });
            v = (double)(T)(v + c * (double)pull_one<L, T, XB>(B, g, p, n, ib));
        }
    }
    return v;
}

template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_force(const T* __restrict__ B, const T* __restrict__ wa,
        const int32_t* __restrict__ lknode, const uint8_t* __restrict__ lkdir,
        const int32_t* __restrict__ lktag, uint32_t n_links, Grid g, Params<L, T> p,
        int n_tags, double* __restrict__ partials) {
    const uint32_t k = blockIdx.x * BX + threadIdx.x;
    double fx = 0, fy = 0, fz = 0;
    int tag = -1;
    if (k < n_links) {
        const int i = lkdir[k];
        const uint32_t n = (uint32_t)lknode[k];
        tag = lktag[k];
        double fp_ib = 0, wi = 0;
        int ex = 0, ey = 0, ez = 0;
        unroll<L::Q>([&](auto I) {
            constexpr int ii = decltype(I)::value;
            if (ii == i) {
                constexpr int ib = TAB<L>.opp[ii];
                fp_ib = (double)ldp<L::Q>(B, ib, n);
                wi = L::W[ii];
                ex = L::E[ii][0];
                ey = L::E[ii][1];
                ez = L::E[ii][2];
            }
        });
        // absolute values: f = delta f + w rho0 (w_i = w_ibar)
        const double v = fp_ib + link_value<L, T, XB>(B, wa, g, p, k, n, i) + 2.0 * wi * p.rho0_d;
        fx = -ex * v;
        fy = -ey * v;
        fz = -ez * v;
    }
    for (int t = 0; t < n_tags; ++t) {
        const bool mine = (tag == t);
        const double comp[3] = {mine ? fx : 0.0, mine ? fy : 0.0, mine ? fz : 0.0};
        for (int a = 0; a < L::D; ++a) {
            const double s = block_sum(comp[a]);
            if (threadIdx.x == 0)
                partials[((size_t)blockIdx.x * n_tags + t) * L::D + a] = s;
        }
    }
}

template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_force_obj(const T* __restrict__ B, const T* __restrict__ wa,
            const int32_t* __restrict__ lknode, const uint8_t* __restrict__ lkdir,
            const int32_t* __restrict__ lktag, uint32_t n_links, Grid g, Params<L, T> p,
            int tag, double weight, double* __restrict__ acc) {
    const uint32_t k = blockIdx.x * BX + threadIdx.x;
    double fx = 0;
    if (k < n_links && lktag[k] == tag) {
        const int i = lkdir[k];
        const uint32_t n = (uint32_t)lknode[k];
        unroll<L::Q>([&](auto I) {
            constexpr int ii = decltype(I)::value;
            if constexpr (L::E[ii][0] != 0) {
                if (ii == i) {
                    constexpr int ib = TAB<L>.opp[ii];
                    const double v = (double)ldp<L::Q>(B, ib, n) +
                                     link_value<L, T, XB>(B, wa, g, p, k, n, ii) +
                                     2.0 * L::W[ii] * p.rho0_d;
                    fx = -L::E[ii][0] * v;
                }
            }
        });
    }
    const double s = block_sum(fx);
    if (threadIdx.x == 0) acc[blockIdx.x] += weight * s;
}

// NaN into n values (debug mode: slots a step leaves unwritten stay NaN)
template <class T>
__global__ void __launch_bounds__(BX) k_fill_nan(T* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * BX;
    for (uint64_t i = (uint64_t)blockIdx.x * BX + threadIdx.x; i < n; i += stride)
        p[i] = (T)__builtin_nan("");
}

// out[c] = sum over rows of partials[row*cols + c]; one block per column,
// fixed summation order
__global__ void __launch_bounds__(BX)
k_sum_blocks(const double* __restrict__ partials, uint32_t rows, uint32_t cols,
             double* __restrict__ out) {
    const uint32_t c = blockIdx.x;
    double s = 0;
    for (uint32_t r = threadIdx.x; r < rows; r += BX) s += partials[(size_t)r * cols + c];
    s = block_sum(s);
    if (threadIdx.x == 0) out[c] = s;
}

// ----------------------------------------------------------------------------
// host side

static Grid make_grid(const Engine& e) {
    Grid g;
    g.nx = (uint32_t)e.nx;
    g.ny = (uint32_t)e.ny;
    g.nz = (uint32_t)e.nz;
    g.N = (uint32_t)e.N;
    g.S = (uint32_t)e.S;
    g.nblocks = (uint32_t)((e.N + BX - 1) / BX);
    g.bpr = e.nx % BX == 0 ? (uint32_t)(e.nx / BX) : 0u;
    return g;
}

unsigned launch_blocks(const Grid& g) { return g.nblocks; }

int64_t step_blocks(const Engine& e) {
    return make_grid(e).nblocks;
}

NodeMeta meta(const Engine& e) { return NodeMeta{e.d_info, e.d_wave}; }
int64_t link_blocks(const Engine& e) { return (e.n_links + BX - 1) / BX; }

template <class L, class T>
static Params<L, T> make_params(const Engine& e) {
    Params<L, T> p;
    for (int k = 0; k < L::Q; ++k) {
        const double r = L::conserved(k) ? 0.0 : e.s[k] / (double)TAB<L>.norm[k];
        p.rate[k] = (T)r;
    }
    for (int a = 0; a < 3; ++a) p.G[a] = (T)(3.0 * e.rho0 * (a < L::D ? e.g[a] : 0.0));
    p.drho = (T)(e.xbc == XBC_PRESSURE ? e.drho : 0.0);
    for (int i = 0; i < L::Q; ++i) {
        double eg = 0;
        for (int a = 0; a < L::D; ++a) eg += L::E[i][a] * e.g[a];
        p.force[i] = (T)(3.0 * L::W[i] * e.rho0 * eg);
        p.seam[i] = (T)(L::W[i] * (e.xbc == XBC_PRESSURE ? e.drho : 0.0));
    }
    p.rho0 = (T)e.rho0;
    p.inv_rho0 = (T)(1.0 / e.rho0);
    p.c0 = 1.0 - e.b;
    p.rho0_d = e.rho0;
    p.wall_scale = e.wall_decay == 1.0 ? 1.0 : e.wall_scale;
    p.c1d = e.two_node ? e.d_lkc1d : nullptr;
    return p;
}

// runtime -> compile-time dispatch over lattice, precision and x boundary
template <class F>
static hipError_t dispatch(const Engine& e, F&& f) {
    auto by_xbc = [&](auto lat, auto prec) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        switch (e.xbc) {
            case XBC_PRESSURE: return f(L{}, T{}, std::integral_constant<int, XBC_PRESSURE>{});
            case XBC_OUTFLOW: return f(L{}, T{}, std::integral_constant<int, XBC_OUTFLOW>{});
            default: return f(L{}, T{}, std::integral_constant<int, XBC_PERIODIC>{});
        }
    };
    if (e.lattice == 0)
        return e.precision == 0 ? by_xbc(D2Q9{}, double{}) : by_xbc(D2Q9{}, float{});
    if (e.lattice == 2)
        return e.precision == 0 ? by_xbc(D3Q15{}, double{}) : by_xbc(D3Q15{}, float{});
    return e.precision == 0 ? by_xbc(D3Q19{}, double{}) : by_xbc(D3Q19{}, float{});
}

hipError_t launch_step(Engine& e, const Snapshot& in, const Snapshot& out,
                       const StepObjective& obj, void* rec) {
    const Grid g = make_grid(e);
    return dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        auto kern = rec ? (g.bpr ? k_step<L, T, XB, true, true> : k_step<L, T, XB, false, true>)
                        : (g.bpr ? k_step<L, T, XB, true, false> : k_step<L, T, XB, false, false>);
        const StepRecord<T> r = rec ? record_at<T>(e, rec) : StepRecord<T>{};
        hipLaunchKernelGGL(kern, dim3(launch_blocks(g)), dim3(BX), 0,
                           e.stream, (const T*)in.f, (T*)out.f, (const T*)in.wa,
                           (T*)out.wa, meta(e), coef_table<T>(e), g,
                           make_params<L, T>(e), obj, r);
        return hipGetLastError();
    });
}

hipError_t launch_init(Engine& e, const double* df, const double* rho,
                       const double* u, const Snapshot& out) {
    const Grid g = make_grid(e);
    return dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_init<L, T, XB>), dim3(launch_blocks(g)), dim3(BX), 0,
                           e.stream, df, rho, u, (T*)out.f, (T*)out.wa, meta(e), g,
                           make_params<L, T>(e));
        return hipGetLastError();
    });
}

hipError_t launch_observe(Engine& e, const Snapshot& in, double* rho, double* u,
                          double* df) {
    const Grid g = make_grid(e);
    return dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_observe<L, T, XB>), dim3(launch_blocks(g)), dim3(BX), 0,
                           e.stream, (const T*)in.f, (const T*)in.wa, meta(e), g,
                           make_params<L, T>(e), rho, u, df);
        return hipGetLastError();
    });
}

hipError_t launch_mass(Engine& e, const Snapshot& in, double* partials,
                       int64_t* nblocks) {
    const Grid g = make_grid(e);
    *nblocks = g.nblocks;
    return dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_mass<L, T, XB>), dim3(launch_blocks(g)), dim3(BX), 0,
                           e.stream, (const T*)in.f, (const T*)in.wa, meta(e), g,
                           make_params<L, T>(e), partials);
        return hipGetLastError();
    });
}

hipError_t launch_plane_density(Engine& e, const Snapshot& in, uint32_t x_in, uint32_t x_out,
                                double a_in, double a_out, double* partials, int64_t* nblocks) {
    const Grid g = make_grid(e);
    const int64_t nb = (2 * e.ny * e.nz + BX - 1) / BX;
    *nblocks = nb;
    return dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_plane_density<L, T, XB>), dim3((unsigned)nb), dim3(BX), 0, e.stream,
                           (const T*)in.f, (const T*)in.wa, meta(e), g, make_params<L, T>(e),
                           x_in, x_out, a_in, a_out, partials);
        return hipGetLastError();
    });
}

hipError_t launch_force(Engine& e, const Snapshot& post, double* partials,
                        int64_t* nblocks) {
    const int64_t nb = link_blocks(e);
    *nblocks = nb;
    if (nb == 0) return hipSuccess;
    const Grid g = make_grid(e);
    return dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_force<L, T, XB>), dim3((unsigned)nb), dim3(BX), 0, e.stream,
                           (const T*)post.f, (const T*)post.wa, e.d_lknode, e.d_lkdir,
                           e.d_lktag, (uint32_t)e.n_links, g, make_params<L, T>(e),
                           e.n_tags, partials);
        return hipGetLastError();
    });
}

hipError_t launch_force_objective(Engine& e, const Snapshot& post, double* acc,
                                  int tag, double weight) {
    const int64_t nb = link_blocks(e);
    if (nb == 0) return hipSuccess;
    const Grid g = make_grid(e);
    return dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_force_obj<L, T, XB>), dim3((unsigned)nb), dim3(BX), 0,
                           e.stream, (const T*)post.f, (const T*)post.wa, e.d_lknode,
                           e.d_lkdir, e.d_lktag, (uint32_t)e.n_links, g,
                           make_params<L, T>(e), tag, weight, acc);
        return hipGetLastError();
    });
}

hipError_t launch_fill_nan(Engine& e, void* p, size_t n) {
    if (n == 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<size_t>((n + BX - 1) / BX, 65536);
    if (e.precision == 0)
        hipLaunchKernelGGL(k_fill_nan<double>, dim3(nb), dim3(BX), 0, e.stream, (double*)p,
                           (uint64_t)n);
    else
        hipLaunchKernelGGL(k_fill_nan<float>, dim3(nb), dim3(BX), 0, e.stream, (float*)p,
                           (uint64_t)n);
    return hipGetLastError();
}

hipError_t launch_sum_blocks(Engine& e, const double* partials, int64_t rows,
                             int64_t cols, double* out) {
    if (cols == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_blocks, dim3((unsigned)cols), dim3(BX), 0, e.stream,
                       partials, (uint32_t)rows, (uint32_t)cols, out);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Fixed device scratch for the entry points that allocate nothing: one array
// per device, held until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host it only names the symbol); it uses the
// device address that hipGetSymbolAddress returns, looked up once per device
// with that device current.

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t st = hipGetDevice(&cur);
        if (st != hipSuccess) return st;
        if (cur != device && (st = hipSetDevice(device)) != hipSuccess) return st;
        void* p = nullptr;
        st = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (st != hipSuccess) return st;
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace lbe
