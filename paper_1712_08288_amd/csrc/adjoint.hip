// Adjoint (reverse-mode) step of the forward kernel.
//
// The forward map of one step t -> t+1 at fluid node y is
//   g(y)   = C(f(y, t))                         collision, Eq. (22a)
//   f_i(y + e_i, t+1) = g_i(y)                  advection, Eq. (22b)
//   f_i(y, t+1) = c0 f_i(y,t) + c1 f_ibar(y,t) + c2 g_i(y) + c3 g_ibar(y)
//                 + c4 * 3 w_i rho0 e_i.phi     cut link (y, i), Eq. (213)
// With lambda(t+1) = dJ/df(., t+1) the reverse step computes, per node,
//   mu_i(y)  = dJ/dg_i(y): lambda_i(y + e_i, t+1) when that node pulls from y,
//              plus c2 / c3 times the node's own link adjoints,
//   lambda(y, t) = (dC/df)^T mu + c0 / c1 times the own link adjoints,
// where (dC/df)^T mu = mu - (I - J^T) M^T R M mu, R = diag(s_k / |M_k|^2),
// and J_ij = d f^eq_i / d f_j = w_i [1 + (3 e_i + 9 (e_i.u) e_i - 3 u).e_j]
// (derivative of Eq. (42)), so that (J^T v)_j = a + b.e_j with
// a = sum_i w_i v_i and b = sum_i w_i v_i (3 e_i + 9 (e_i.u) e_i - 3 u).
// Gradients accumulated on the way, in double (the per-link ones by the
// lanes that carry the links, the others in per-block sums):
//   dJ/dgamma_k += a_k (dc1 f_ibar + dc2 g_i + dc3 g_ibar + ws dwall),
//   dJ/dphi_k   += a_k ws c4 3 w_i rho0 e_i,
//   dJ/dg       += sum_i mu_i 3 w_i rho0 e_i,
//   dJ/ds_k     += -(M mu)_k (M (f - f^eq))_k / |M_k|^2,
// where a_k is the adjoint of the link value f_i(y, t+1) and ws the
// wall-data factor of step t.  The wall terms share the factor a_k ws, so
// per link only two sums are kept, gq_k = sum a_k (dc1 f_ibar + dc2 g_i +
// dc3 g_ibar) and gs_k = sum a_k ws; the gradients are formed from them
// when read (k_link_finish).
#include "engine.hpp"
#include "kernels.hpp"

namespace lbe {

// Node indices of x + e (the node that pulls from this one along e).
template <int XB>
struct Push {
    uint32_t xt[3];
    uint32_t row[3][3];
    bool x_out;   // outflow: no node at x = nx (e_x = +1 from the last column)

    __device__ __forceinline__ Push(const Grid& g, const NodePos& p) {
        const uint32_t xm = p.ix == 0 ? g.nx - 1 : p.ix - 1;
        const uint32_t xp = p.ix + 1 == g.nx ? 0u : p.ix + 1;
        xt[0] = xm;       // e_x = -1 lands at x - 1
        xt[1] = p.ix;
        xt[2] = xp;       // e_x = +1 lands at x + 1
        x_out = (XB == XBC_OUTFLOW) && (p.ix + 1 == g.nx);
        const uint32_t ys[3] = {p.iy == 0 ? g.ny - 1 : p.iy - 1, p.iy,
                                p.iy + 1 == g.ny ? 0u : p.iy + 1};
        const uint32_t zs[3] = {p.iz == 0 ? g.nz - 1 : p.iz - 1, p.iz,
                                p.iz + 1 == g.nz ? 0u : p.iz + 1};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) row[a][c] = g.nx * (ys[a] + g.ny * zs[c]);
    }

    template <class L, int I>
    __device__ __forceinline__ uint32_t dst() const {
        return xt[L::E[I][0] + 1] + row[L::E[I][1] + 1][L::E[I][2] + 1];
    }
    // outflow: the last column also pulls its -x populations from here
    template <class L, int I>
    __device__ __forceinline__ uint32_t dst_clamped(uint32_t ix) const {
        return ix + row[L::E[I][1] + 1][L::E[I][2] + 1];
    }
};

struct AdjArgs {
    int obj_kind;        // LBM_OBJ_* of the header
    int obj_tag;
    double w_force;      // weight of this step's drag term (0 outside window)
    double w_ux;         // weight of d(mean u_x)/df_j = e_jx * w_ux
    int want_ds;
    // pressure drop: dJ/df_j(x) = a_in [x = x_in] - a_out [x = x_out] for
    // every j at fluid nodes (a_* include the step's weight and c_s^2)
    uint32_t x_in, x_out;
    double a_in, a_out;
};

// The per-link gradient sums of the sweep (see the header): gq at g[k] and
// gs at g[L1 + k], with the gamma-derivatives of the coefficients they
// need.  In the kernel that reads step records g is instead the step's run
// of a_k (one per link), summed later by k_link_sums.  Pointers are few on
// purpose: every kernel argument the adjoint keeps costs scalar registers,
// which bound its occupancy.
struct LinkGrad {
    const LinkDeriv* deriv;
    double* g;
    uint32_t L1;     // max(L, 1): the stride of the runs of g and of a record
};

// One step's contribution of link k with adjoint a_k (drag term included)
// and the forward values f_ibar(y, t), f'_i(y, t), f'_ibar(y, t).
template <class T>
__device__ __forceinline__ void link_gradient(const LinkGrad& lg, uint32_t k, double ak, T fib,
                                              T fpi, T fpib, double ws) {
    const double d1 = lg.deriv[k].d1, d2 = lg.deriv[k].d2, d3 = lg.deriv[k].d3;
    lg.g[k] += ak * (d1 * (double)fib + d2 * (double)fpi + d3 * (double)fpib);
    lg.g[lg.L1 + k] += ak * ws;
}
// The same with the three forward values read from the link runs of a step
// record (fib at lk[k], f'_i at lk[L1 + k], f'_ibar at lk[2 L1 + k]).
template <class T>
__device__ __forceinline__ void link_gradient_rec(const LinkGrad& lg, const T* __restrict__ lk,
                                                  uint32_t k, double ak, double ws) {
    link_gradient(lg, k, ak, lk[k], lk[lg.L1 + k], lk[2 * lg.L1 + k], ws);
}

// The pending reverse steps on records: step j's a_k run at ak[j L1], the
// link runs of its record at lk[j] and its wall-data factor ws[j], in the
// order the steps were taken.
template <class T>
struct AkBatch {
    const T* lk[kAkBatch];
    double ws[kAkBatch];
    int count;
};

// Their terms added to the two sums of every link, step by step in that
// order (the same additions, in the same order, as one step at a time):
// one thread per link, the sums and the coefficient derivatives read once.
// tq (Eq. (211) runs, else null): the pre-pass's gq term of each step, in
// the layout of ak.
template <class T>
__global__ void __launch_bounds__(BX)
k_link_sums(const double* __restrict__ ak, const double* __restrict__ tq, AkBatch<T> b,
            LinkGrad lg, uint32_t L) {
    const uint32_t k = blockIdx.x * BX + threadIdx.x;
    if (k >= L) return;
    const double d1 = lg.deriv[k].d1, d2 = lg.deriv[k].d2, d3 = lg.deriv[k].d3;
    double gq = lg.g[k], gs = lg.g[lg.L1 + k];
    for (int j = 0; j < b.count; ++j) {
        // Eq. (211): the pre-pass's term of step j comes first, as when the
        // pre-pass added it itself
        if (tq) gq += tq[(size_t)j * lg.L1 + k];
        const double a = ak[(size_t)j * lg.L1 + k];
        const T* __restrict__ lk = b.lk[j];
        gq += a * (d1 * (double)lk[k] + d2 * (double)lk[lg.L1 + k] +
                   d3 * (double)lk[2 * lg.L1 + k]);
        gs += a * b.ws[j];
    }
    lg.g[k] = gq;
    lg.g[lg.L1 + k] = gs;
}

// Walk a node's cut links in direction order (links are sorted by node,
// then direction, so the k-th set bit of the mask is link nl.base + k).  For
// the wave's first 64 links the two LDS values of the link, st.v[A][k] and
// st.v[B][k], are read one direction ahead of their use, with the index
// clamped to the slab instead of a divergent branch around the access, so
// that the reads overlap; own(I, va, vb, k) consumes them, direct(I, k)
// handles a link past the 64th.
template <class L, class T, int A, int B, class Own, class Direct>
__device__ __forceinline__ void walk_links(const NodeLinks& nl, LinkStage<T>& st, Own&& own,
                                           Direct&& direct) {
    uint32_t k = nl.base;
    uint32_t kk = k < 64u ? k : 63u;
    T a_next = st.v[A][kk], b_next = st.v[B][kk];
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (i > 0) {
            const uint32_t bit = (nl.mask >> i) & 1u;
            const T va = a_next, vb = b_next;
            const uint32_t k1 = k + bit;
            if constexpr (i + 1 < L::Q) {
                kk = k1 < 64u ? k1 : 63u;
                a_next = st.v[A][kk];
                b_next = st.v[B][kk];
            }
            if (bit) {
                if (k < 64u) own(I, va, vb, k);
                else direct(I, k);
            }
            k = k1;
        }
    });
}

template <int NC>
__device__ __forceinline__ void block_accumulate(const double (&v)[NC], double* __restrict__ dst) {
    __shared__ double part[BX / 64][NC];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double x = v[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
        if (lane == 0) part[wid][c] = x;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        double s = 0;
        for (int w = 0; w < BX / 64; ++w) s += part[w][threadIdx.x];
        dst[threadIdx.x] += s;
    }
}

// Lattice data of a direction known only at run time (link lanes): e_d, w_d
// and the opposite direction.
template <class L>
__device__ __forceinline__ void dir_data(int d, int (&e)[3], double& w, int& opp) {
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (i == d) {
            e[0] = L::E[i][0];
            e[1] = L::E[i][1];
            e[2] = L::E[i][2];
            w = L::W[i];
            opp = TAB<L>.opp[i];
        }
    });
}

// Link k = (y, i) of a mixed wave, handled by the lane of its node y: the
// contribution of its adjoint a_k to mu and to lambda(y, t), and its
// gradient sums (forward values from the step record when UM, else from
// the pulled state and the state at t + 1).  Used for links past the 64th
// of a wave (the first 64 go through the wave's LDS slab).
template <class L, class T, int i, bool UM>
__device__ __forceinline__ void own_link_direct(uint32_t k, const T* __restrict__ lam_in,
                                                const T* __restrict__ nxt,
                                                const StepRecord<T>& rec, uint32_t n,
                                                const LinkCoefT<T>* __restrict__ lkcoef,
                                                const int32_t* __restrict__ lktag,
                                                const LinkGrad& lgr,
                                                const Params<L, T>& p, const AdjArgs& a,
                                                const T (&f)[L::Q], T (&mu)[L::Q]) {
    constexpr int ib = TAB<L>.opp[i];
    double ak = (double)ldp<L::Q>(lam_in, i, n);
    if (a.obj_kind == 1 && L::E[i][0] != 0 && lktag[k] == a.obj_tag) {
        // drag: (e_ibar)_x (f'_ibar(y,t) + f_i(y,t+1))
        const double dfx = -(double)L::E[i][0] * a.w_force;
        ak += dfx;
        mu[ib] += (T)dfx;
    }
    const LinkCoefT<T> c = lkcoef[k];
    mu[i] += (T)(c.c2 * ak);
    mu[ib] += (T)(c.c3 * ak);
    if constexpr (UM)
        lgr.g[k] = ak;   // the step's a_k run; k_link_sums adds the terms
    else
        link_gradient(lgr, k, ak, f[ib], ldp<L::Q>(nxt, i, n), ldp<L::Q>(nxt, ib, n),
                      p.wall_scale);
}

// The terms of such a link that bypass the collision: c0 a_k onto
// lambda_i(y, t) and c1 a_k onto lambda_ibar(y, t), added to mu after its
// moments are taken (a_k read again: these links are rare).
template <class L, class T, int i>
__device__ __forceinline__ void own_link_bypass(uint32_t k, const T* __restrict__ lam_in,
                                                uint32_t n,
                                                const LinkCoefT<T>* __restrict__ lkcoef,
                                                const int32_t* __restrict__ lktag,
                                                const Params<L, T>& p, const AdjArgs& a,
                                                T (&mu)[L::Q]) {
    constexpr int ib = TAB<L>.opp[i];
    double ak = (double)ldp<L::Q>(lam_in, i, n);
    if (a.obj_kind == 1 && L::E[i][0] != 0 && lktag[k] == a.obj_tag)
        ak += -(double)L::E[i][0] * a.w_force;
    mu[i] += (T)(p.c0 * ak);
    mu[ib] += (T)(lkcoef[k].c1 * ak);
}

// The gradients of every link from its two sums, in the caller's link
// order: dq[perm k] = gq_k + dwall_k gs_k and
// dphi[perm k][a] = c4_k 3 w_i rho0 e_ia gs_k (either output may be null).
template <class L>
__global__ void __launch_bounds__(BX)
k_link_finish(const double* __restrict__ gq, const double* __restrict__ gs,
              const LinkDeriv* __restrict__ deriv, const double* __restrict__ lkc4,
              const uint8_t* __restrict__ lkdir, const int32_t* __restrict__ perm,
              double rho0, uint32_t n_links, double* __restrict__ dq,
              double* __restrict__ dphi) {
    const uint32_t k = blockIdx.x * BX + threadIdx.x;
    if (k >= n_links) return;
    const size_t pk = (size_t)(uint32_t)perm[k];
    if (dq) dq[pk] = gq[k] + deriv[k].dwall * gs[k];
    if (dphi) {
        int e[3] = {0, 0, 0}, ib = 0;
        double w = 0.0;
        dir_data<L>(lkdir[k], e, w, ib);
        const double c = lkc4[k] * 3.0 * w * rho0 * gs[k];
#pragma unroll
        for (int al = 0; al < L::D; ++al) dphi[pk * L::D + al] = c * e[al];
    }
}

// The waves of the adjoint launch, slot s < count (s = 4 blockIdx.x + wave in
// the block), each as {id, kind | links << 2, first link, 0} (node
// n = 64 id + lane) so that one scalar load brings all of it.  wpr = nx / 64
// when 64 divides nx (each wave lies in one row), else 0.
struct WaveList {
    const uint4* ent;
    uint32_t count;
    uint32_t wpr;
};

template <bool ROWS>
__device__ __forceinline__ NodePos node_of_wave(const Grid& g, const WaveList& wl, uint32_t w,
                                                uint32_t lane, bool active) {
    NodePos p;
    p.n = w * 64u + lane;
    p.in = active && p.n < g.N;
    if constexpr (ROWS) {
        const uint32_t row = w / wl.wpr;
        p.ix = (w - row * wl.wpr) * 64u + lane;
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

// One launch covers the non-idle waves in memory order.  Plain and mixed
// waves take separate paths from the start.  Mixed waves handle their cut
// links cooperatively (see LinkStage): the link lanes read the link data
// and a_k = lambda_i(y, t+1) (plus the drag term) with coalesced loads and
// hand c2 a_k, c3 a_k (+ drag), c0 a_k and c1 a_k to the node's lane
// through LDS; the node's lane hands back f_ibar(y, t), from which with
// a_k and the forward step's stored f'_i(y, t), f'_ibar(y, t) the link
// lanes add the link's gradient sums.
// UM: the forward state enters the collision adjoint only through its
// velocity (the equilibrium's Jacobian depends on u alone), so with the rate
// gradients off the kernel reads u(y, t) recorded by the forward step (D
// planes of U) instead of pulling the Q populations of f(y, t), and the
// link values of the gradients come from the same step record: A, wa and
// nxt are not read.
// FP64 on step records asks for 4 waves per SIMD: the kernel needs 130
// VGPRs, and fitting 128 (two values spilled to scratch) made the reverse
// step 3.5% faster at 256^3; the other variants are left to the compiler
// (forcing more waves on them spilled more and was slower).
template <class L, class T, int XB, bool WANT_DS, bool ROWS, bool UM>
__global__ void __launch_bounds__(BX)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 && UM ? 4 : 1)))
k_adjoint(const T* __restrict__ A, StepRecord<T> rec, const T* __restrict__ wa,
          const T* __restrict__ nxt,
          const T* __restrict__ lam_in, T* __restrict__ lam_out,
          NodeMeta nm, WaveList wl, const LinkCoefT<T>* __restrict__ lkcoef,
          const int32_t* __restrict__ lktag,
          const uint8_t* __restrict__ lkdir, const int32_t* __restrict__ lknode,
          LinkGrad lgr, double* __restrict__ gglob, Grid g, Params<L, T> p, AdjArgs a) {
    constexpr int Q = L::Q, D = L::D, NP = NPAIR<L>;
    static_assert(!(UM && WANT_DS), "the rate gradients need the forward populations");
    constexpr int NC = D + Q;                 // layout of the per-block sums
    constexpr int NR = WANT_DS ? NC : D;      // columns reduced here
    __shared__ LinkStage<T> stage[BX / 64];
    // the link lanes' a_k, parked while the node's work runs (registers are
    // scarcest there)
    __shared__ double ak_park[BX / 64][64];
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t slot = blockIdx.x * (BX / 64) + wid;
    const bool active = slot < wl.count;
    const uint4 wm = active ? wl.ent[slot] : uint4{0u, 0u, 0u, 0u};
    const uint32_t w = __builtin_amdgcn_readfirstlane(wm.x);
    const uint32_t wx = __builtin_amdgcn_readfirstlane(wm.y);
    const uint32_t nlw = wave_links(uint2{wx, 0u});
    const uint32_t wbase = __builtin_amdgcn_readfirstlane(wm.z);
    const NodePos pos = node_of_wave<ROWS>(g, wl, w, lane, active);
    LinkStage<T>& st = stage[wid];
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;

    // One wave's work.  Plain and mixed waves take separate paths from the
    // start (their own loads included), so that each path's registers are
    // allocated as in a kernel of its own.  Plain waves are 64 fluid nodes
    // inside the grid.
    auto run = [&](auto mixed_c) {
        constexpr bool MX = decltype(mixed_c)::value;
        // mixed waves: the link lanes' indices come first (small coalesced
        // loads), so that the gathers that depend on them can be issued before
        // the node loads below return
        const bool link_lane = MX && lane < nlw && lane < 64u;
        const uint32_t kl = wbase + lane;
        int ld_dir = 0;
        uint32_t ld_node = 0;
        if (link_lane) {
            ld_dir = lkdir[kl];
            ld_node = (uint32_t)lknode[kl];
        }

        // loads that do not depend on the node's metadata: the planes of the
        // forward pull and the adjoint gathers lambda_i(y + e_i, t+1) (entries
        // of solid or absent neighbours are read and then discarded)
        T f[Q], lg[Q], uv[3] = {T(0), T(0), T(0)};
        const Push<XB> ps(g, pos);
        // plain waves are 64 fluid nodes inside the grid; in mixed waves the
        // lanes of 64-byte plane segments without fluid nodes neither read nor
        // write
        const bool live = !MX || (pos.in && lane_in_live_segment<T>(wx, lane));
        if (live) {
            if constexpr (UM) {
                for (int a = 0; a < D; ++a) uv[a] = ld(rec.u + (size_t)a * g.S, pos.n);
            } else {
                pull_planes<L, T, XB>(A, g, pos, p, NodeLinks{0u, 0u}, f);
            }
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                lg[i] = ldp<Q>(lam_in, i, i == 0 ? pos.n : ps.template dst<L, i>());
            });
        } else {
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                f[i] = T(0);
                lg[i] = T(0);
            });
        }

        // one fluid node; PLAIN: the whole wave is fluid without cut links.  In
        // a mixed wave nl.base is relative to the wave's first link and f already
        // holds the link slots.
        auto node = [&](auto plain_c, const NodeLinks& nl) {
            constexpr bool PLAIN = decltype(plain_c)::value;
            // forward state f(y, t) and its velocity (UM: the recorded one)
            T sp[NP], dp[NP];
            T rho = 0, j[3] = {0, 0, 0}, u[3];
            if constexpr (UM) {
                u[0] = uv[0];
                u[1] = uv[1];
                u[2] = uv[2];
            } else {
                pair_split<L, T>(f, sp, dp);
                conserved_of<L, T>(f[0], sp, dp, rho, j);
                u[0] = j[0] * p.inv_rho0;
                u[1] = j[1] * p.inv_rho0;
                u[2] = j[2] * p.inv_rho0;
            }

            // mu_i(y) = dJ/df'_i(y): lambda_i(y + e_i, t+1) where that node pulls
            T mu[Q];
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int ib = TAB<L>.opp[i];
                if constexpr (i == 0) {
                    mu[i] = lg[0];
                } else {
                    bool lost = (nl.mask >> ib) & 1u;     // y + e_i is solid
                    if constexpr (XB == XBC_OUTFLOW && L::E[i][0] == 1) lost = lost || ps.x_out;
                    mu[i] = lost ? T(0) : lg[i];
                    if constexpr (XB == XBC_OUTFLOW && L::E[i][0] == -1) {
                        if (ps.x_out) {
                            const uint32_t n2 = ps.template dst_clamped<L, i>(pos.ix);
                            if (!is_solid(nm.info[n2])) mu[i] += ldp<Q>(lam_in, i, n2);
                        }
                    }
                }
            });

            // own cut links: Eq. (213) reversed and the drag terms; f_ibar(y, t)
            // goes back to the link lane (the gradients are taken per link)
            if constexpr (!PLAIN) {
                if (nl.mask) {
                    walk_links<L, T, 0, 1>(
                        nl, st,
                        [&](auto I, T va, T vb, uint32_t k) {
                            constexpr int i = decltype(I)::value;
                            constexpr int ib = TAB<L>.opp[i];
                            mu[i] += va;
                            mu[ib] += vb;
                            if constexpr (!UM) st.v[0][k] = f[ib];
                        },
                        [&](auto I, uint32_t k) {
                            constexpr int i = decltype(I)::value;
                            own_link_direct<L, T, i, UM>(wbase + k, lam_in, nxt, rec, pos.n,
                                                         lkcoef, lktag, lgr, p, a, f, mu);
                        });
                }
            }

            // collision adjoint: lambda = mu - v + J^T v + (c0, c1 link terms),
            // v = M^T R M mu
            T smu[NP], dmu[NP];
            pair_split<L, T>(mu, smu, dmu);
            T qm[Q];
            moments_of<L, T>(mu[0], smu, dmu, qm);

            // dJ/dg += 3 rho0 sum_i w_i e_i mu_i (pair form: w_i e_i (mu_i - mu_ibar)),
            // summed over the node in T, accumulated over nodes in double
            // (taken here in mixed waves, so that dmu dies before the link
            // terms below; at the end in plain waves)
            auto add_dg = [&]() {
                T sg3[3] = {0, 0, 0};
                unroll<NP>([&](auto P) {
                    constexpr int pp = decltype(P)::value;
                    constexpr int i = DER<L>.pi[pp];
                    const T t = T(L::W[i]) * dmu[pp];
                    macc<L::E[i][0]>(sg3[0], t);
                    macc<L::E[i][1]>(sg3[1], t);
                    macc<L::E[i][2]>(sg3[2], t);
                });
#pragma unroll
                for (int al = 0; al < D; ++al) acc[al] += 3.0 * p.rho0_d * (double)sg3[al];
            };
            if constexpr (!PLAIN) add_dg();

            // the link terms that bypass the collision (c0 a_k onto
            // lambda_i(y, t), c1 a_k onto lambda_ibar(y, t)) join mu now that
            // its moments are taken, so that they need no registers of their own
            if constexpr (!PLAIN) {
                if (nl.mask) {
                    walk_links<L, T, 2, 3>(
                        nl, st,
                        [&](auto I, T va, T vb, uint32_t) {
                            constexpr int i = decltype(I)::value;
                            constexpr int ib = TAB<L>.opp[i];
                            mu[i] += va;
                            mu[ib] += vb;
                        },
                        [&](auto I, uint32_t k) {
                            constexpr int i = decltype(I)::value;
                            own_link_bypass<L, T, i>(wbase + k, lam_in, pos.n, lkcoef, lktag, p,
                                                     a, mu);
                        });
                }
            }
            T r[Q];
            unroll<Q>([&](auto K) {
                constexpr int kk = decltype(K)::value;
                r[kk] = L::conserved(kk) ? T(0) : qm[kk] * p.rate[kk];
            });
            T e0, ev[NP], od[NP];
            back_transform<L, T>(r, e0, ev, od);
            // J^T v = as + b.e_j with as = sum w_i v_i and
            // b = sum_i w_i v_i (3 e_i + 9 (e_i.u) e_i) - 3 u as
            T as = T(L::W[0]) * e0;
            T b[3] = {0, 0, 0};
            unroll<NP>([&](auto P) {
                constexpr int pp = decltype(P)::value;
                constexpr int i = DER<L>.pi[pp];
                const T w2 = T(2.0 * L::W[i]);
                as += w2 * ev[pp];
                T eu = 0;
                macc<L::E[i][0]>(eu, u[0]);
                macc<L::E[i][1]>(eu, u[1]);
                macc<L::E[i][2]>(eu, u[2]);
                const T t = w2 * (T(3) * od[pp] + T(9) * eu * ev[pp]);
                macc<L::E[i][0]>(b[0], t);
                macc<L::E[i][1]>(b[1], t);
                macc<L::E[i][2]>(b[2], t);
            });
            b[0] -= T(3) * u[0] * as;
            b[1] -= T(3) * u[1] * as;
            b[2] -= T(3) * u[2] * as;
            const T wux = (T)a.w_ux;
            // pressure drop: the same term for every population of the node
            if (a.obj_kind == 3)
                as += (T)((pos.ix == a.x_in ? a.a_in : 0.0) - (pos.ix == a.x_out ? a.a_out : 0.0));
            auto finish = [&](auto J, T v) {
                constexpr int jd = decltype(J)::value;
                T out = mu[jd] - v + as;
                macc<L::E[jd][0]>(out, b[0]);
                macc<L::E[jd][1]>(out, b[1]);
                macc<L::E[jd][2]>(out, b[2]);
                if (a.obj_kind == 2) macc<L::E[jd][0]>(out, wux);
                stp_nt<Q>(lam_out, jd, pos.n, out);
            };
            finish(std::integral_constant<int, 0>{}, e0);
            unroll<NP>([&](auto P) {
                constexpr int pp = decltype(P)::value;
                constexpr int i = DER<L>.pi[pp];
                constexpr int ib = TAB<L>.opp[i];
                finish(std::integral_constant<int, i>{}, ev[pp] + od[pp]);
                finish(std::integral_constant<int, ib>{}, ev[pp] - od[pp]);
            });
            if constexpr (PLAIN) add_dg();
            if constexpr (WANT_DS) {
                // dJ/ds_k -= (M mu)_k (M (f - f^eq))_k / |M_k|^2
                T m[Q];
                moments_of<L, T>(f[0], sp, dp, m);
                subtract_equilibrium<L, T>(m, rho, j, p.inv_rho0);
                unroll<Q>([&](auto K) {
                    constexpr int kk = decltype(K)::value;
                    if constexpr (!L::conserved(kk))
                        acc[D + kk] -= (double)qm[kk] * (double)m[kk] / (double)TAB<L>.norm[kk];
                });
            }
        };

        if constexpr (!MX) {
            node(std::true_type{}, NodeLinks{0u, 0u});
        } else {
            // link lanes: the link's adjoint a_k = lambda_i(y, t+1) and (reading
            // states) the forward step's stored f'_i(y, t), f'_ibar(y, t)
            int le[3] = {0, 0, 0}, lib = 0;
            double lw = 0.0;
            double ak = 0.0;
            T fpi = T(0), fpib = T(0);
            LinkCoefT<T> c{T(0), T(0), T(0), T(0)};
            if (link_lane) {
                dir_data<L>(ld_dir, le, lw, lib);
                c = lkcoef[kl];
                ak = (double)ldp<Q>(lam_in, ld_dir, ld_node);
                if constexpr (!UM) {
                    fpi = ldp<Q>(nxt, ld_dir, ld_node);
                    fpib = ldp<Q>(nxt, lib, ld_node);
                }
            }
            const uint32_t info = live ? nm.info[pos.n] : kInfoSolid;
            const bool sol = is_solid(info);
            const NodeLinks nl = sol ? NodeLinks{0u, 0u} : node_links(info, 0u);
            if constexpr (!UM) {
                // forward state: the link slots of the recorded step
                const T wa0 = lane < nlw ? wa[wbase + lane] : T(0);
                wave_link_values<L, T>(wa, wbase, lane, wa0, nl, st, f);
                if (p.c1d) complete_two_node<L, T>(p.c1d + wbase, nl, f);
            }
            // link lanes: the pieces of mu and lambda(y, t) that a_k feeds
            if (link_lane) {
                double dfx = 0.0;
                if (a.obj_kind == 1 && le[0] != 0 && lktag[kl] == a.obj_tag) {
                    // drag: (e_ibar)_x (f'_ibar(y,t) + f_i(y,t+1))
                    dfx = -(double)le[0] * a.w_force;
                    ak += dfx;
                }
                st.v[0][lane] = (T)(c.c2 * ak);
                st.v[1][lane] = (T)(c.c3 * ak + dfx);
                st.v[2][lane] = (T)(p.c0 * ak);
                st.v[3][lane] = (T)(c.c1 * ak);
                // the link's gradient sums: with records a_k is stored into the
                // step's run and k_link_sums adds the terms; else they are added
                // once the node's lane has handed back f_ibar(y, t)
                if constexpr (UM)
                    lgr.g[kl] = ak;
                else
                    ak_park[wid][lane] = ak;
            }
            wave_lds_sync();
            if (!sol) node(std::false_type{}, nl);
            wave_lds_sync();
            if constexpr (!UM)
                if (link_lane)
                    link_gradient(lgr, kl, ak_park[wid][lane], st.v[0][lane], fpi, fpib,
                                  p.wall_scale);
            // the solid lanes store NaN (nothing reads lambda at solid nodes) so
            // that the wave writes whole lines of lam_out: partial lines cost
            // HBM read-modify-write cycles
            if (live && sol) {
                unroll<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    stp_nt<Q>(lam_out, i, pos.n, (T)__builtin_nan(""));
                });
            }
        }
    };
    if (active) {
        if ((__builtin_amdgcn_readfirstlane(wm.y) & 3u) == WAVE_PLAIN)
            run(std::false_type{});
        else
            run(std::true_type{});
    }

    // every wave of the block reaches the barrier inside
    block_accumulate<NR>(acc, gglob + (size_t)blockIdx.x * NC);
}

// Eq. (211) links k = (x_f, i) with a deferred c1: the link value is
// f_i(x_f, t+1) = (terms at t) + c1 f_ibar(x_f, t+1), so its adjoint a_k also
// reaches f_ibar(x_f, t+1) (whose own adjoint the node x_f + e_i gathers in
// the next kernel) and dJ/dgamma gets a_k dc1 f_ibar(x_f, t+1).  That value
// is pulled from the state at t+1 (A_next), or read from fib_next (the
// link values of the step record of t+1, or of the run's final state).
template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_two_node_pre(const T* __restrict__ A_next, const T* __restrict__ fib_next,
               T* __restrict__ lam_in,
               const int32_t* __restrict__ lknode, const uint8_t* __restrict__ lkdir,
               const int32_t* __restrict__ lktag, const double* __restrict__ c1d,
               const double* __restrict__ d1d, double* __restrict__ gq, int store,
               uint32_t n_links, Grid g, Params<L, T> p, AdjArgs a) {
    const uint32_t k = blockIdx.x * BX + threadIdx.x;
    if (k >= n_links) return;
    const double c = c1d[k];
    if (c == 0.0) {
        if (store) gq[k] = 0.0;
        return;
    }
    const int i = lkdir[k];
    const uint32_t n = (uint32_t)lknode[k];
    int ib = 0, ex = 0;
    unroll<L::Q>([&](auto I) {
        constexpr int ii = decltype(I)::value;
        if (ii == i) {
            ib = TAB<L>.opp[ii];
            ex = L::E[ii][0];
        }
    });
    double ak = (double)ldp<L::Q>(lam_in, i, n);
    if (a.obj_kind == 1 && ex != 0 && lktag[k] == a.obj_tag) ak += -(double)ex * a.w_force;
    T* dst = lam_in + pop_at<L::Q>(ib, n);
    *dst = (T)((double)*dst + c * ak);
    const T fib = fib_next ? fib_next[k] : pull_one<L, T, XB>(A_next, g, p, n, ib);
    // store: the step's run of terms that k_link_sums adds (record sweeps)
    if (store)
        gq[k] = ak * d1d[k] * (double)fib;
    else
        gq[k] += ak * d1d[k] * (double)fib;
}

// The value f_ibar(x_f, t) that the pull of the opposite direction reads at
// each link's node from the state A (for Eq. (211) links the plain pull:
// their opposite direction is no cut link), into out[k].
template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_link_pull(const T* __restrict__ A, const int32_t* __restrict__ lknode,
            const uint8_t* __restrict__ lkdir, uint32_t n_links, Grid g, Params<L, T> p,
            T* __restrict__ out) {
    const uint32_t k = blockIdx.x * BX + threadIdx.x;
    if (k >= n_links) return;
    int ib = 0;
    const int i = lkdir[k];
    unroll<L::Q>([&](auto I) {
        constexpr int ii = decltype(I)::value;
        if (ii == i) ib = TAB<L>.opp[ii];
    });
    out[k] = pull_one<L, T, XB>(A, g, p, (uint32_t)lknode[k], ib);
}

template <class L, class T>
__global__ void __launch_bounds__(BX)
k_adjoint_out(const T* __restrict__ lam, const uint32_t* __restrict__ info,
              uint32_t N, double* __restrict__ out) {
    const uint32_t n = blockIdx.x * BX + threadIdx.x;
    if (n >= N) return;
    const bool fluid = !is_solid(info[n]);
    for (int i = 0; i < L::Q; ++i)
        out[(size_t)i * N + n] = fluid ? (double)ldp<L::Q>(lam, i, n) : 0.0;
}

// ----------------------------------------------------------------------------

template <class L, class T>
static Params<L, T> adj_params(const Engine& e) {
    Params<L, T> p;
    for (int k = 0; k < L::Q; ++k)
        p.rate[k] = (T)(L::conserved(k) ? 0.0 : e.s[k] / (double)TAB<L>.norm[k]);
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

static Grid adj_grid(const Engine& e) {
    Grid g;
    g.nx = (uint32_t)e.nx;
    g.ny = (uint32_t)e.ny;
    g.nz = (uint32_t)e.nz;
    g.N = (uint32_t)e.N;
    g.S = (uint32_t)e.S;
    // the adjoint kernels index waves and links, not blocks of a node launch
    g.nblocks = (uint32_t)((e.N + BX - 1) / BX);
    g.bpr = 0u;
    return g;
}

template <class F>
static hipError_t adj_dispatch(const Engine& e, F&& f) {
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

static uint32_t wave_blocks(int64_t waves) { return (uint32_t)((waves + BX / 64 - 1) / (BX / 64)); }

int64_t adjoint_blocks(const Engine& e) {
    return std::max<int64_t>(1, (int64_t)wave_blocks(e.n_wact));
}

hipError_t launch_adjoint_step(Engine& e, const Snapshot* fwd, const Snapshot* next,
                               const void* rec, const void* lam_in, void* lam_out,
                               const AdjointObjective& obj) {
    const Grid g = adj_grid(e);
    const uint32_t wpr = e.nx % 64 == 0 ? (uint32_t)(e.nx / 64) : 0u;
    const WaveList waves{e.d_wact, (uint32_t)e.n_wact, wpr};
    AdjArgs a;
    a.obj_kind = obj.kind;
    a.obj_tag = obj.tag;
    a.w_force = obj.kind == 1 ? obj.weight : 0.0;
    a.w_ux = obj.kind == 2 ? obj.weight * obj.inv_nfluid / e.rho0 : 0.0;
    a.want_ds = e.want_ds ? 1 : 0;
    a.x_in = obj.x_in;
    a.x_out = obj.x_out;
    a.a_in = obj.kind == 3 ? obj.weight * obj.a_in / 3.0 : 0.0;
    a.a_out = obj.kind == 3 ? obj.weight * obj.a_out / 3.0 : 0.0;
    return adj_dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        const bool um = rec != nullptr && !a.want_ds;
        if (!um && (!fwd || !next)) return hipErrorInvalidValue;
        auto kern = a.want_ds ? (wpr ? k_adjoint<L, T, XB, true, true, false>
                                     : k_adjoint<L, T, XB, true, false, false>)
                    : um      ? (wpr ? k_adjoint<L, T, XB, false, true, true>
                                     : k_adjoint<L, T, XB, false, false, true>)
                              : (wpr ? k_adjoint<L, T, XB, false, true, false>
                                     : k_adjoint<L, T, XB, false, false, false>);
        const Params<L, T> prm = adj_params<L, T>(e);
        const StepRecord<T> r = um ? record_at<T>(e, rec) : StepRecord<T>{};
        const size_t L1 = (size_t)std::max<int64_t>(e.n_links, 1);
        if (um && !e.ak_buf) return hipErrorInvalidValue;
        if (um && e.ak_pending == kAkBatch) {
            const hipError_t fs = launch_link_sums(e);
            if (fs != hipSuccess) return fs;
        }
        const LinkGrad lgr{e.d_lkderiv, um ? e.ak_buf + (size_t)e.ak_pending * L1 : e.d_gq,
                           (uint32_t)L1};
        if (waves.count)
            hipLaunchKernelGGL(kern, dim3(wave_blocks(waves.count)), dim3(BX), 0, e.stream,
                               um ? nullptr : (const T*)fwd->f, r,
                               um ? nullptr : (const T*)fwd->wa, um ? nullptr : (const T*)next->f,
                               (const T*)lam_in, (T*)lam_out,
                               NodeMeta{e.d_info, e.d_wave}, waves, coef_table<T>(e),
                               e.d_lktag, e.d_lkdir, e.d_lknode, lgr,
                               e.d_gglob, g, prm, a);
        const hipError_t st = hipGetLastError();
        if (st != hipSuccess || !um || !e.n_links) return st;
        // a link with no fluid node in an active wave cannot exist, so every
        // a_k of the run was written
        e.ak_rec[e.ak_pending] = rec;
        e.ak_ws[e.ak_pending] = e.wall_scale;
        ++e.ak_pending;
        return hipSuccess;
    });
}

hipError_t launch_link_sums(Engine& e) {
    if (e.ak_pending == 0) return hipSuccess;
    const int count = e.ak_pending;
    e.ak_pending = 0;
    const uint32_t L1 = (uint32_t)std::max<int64_t>(e.n_links, 1);
    const LinkGrad lgr{e.d_lkderiv, e.d_gq, L1};
    const unsigned nb = (unsigned)((e.n_links + BX - 1) / BX);
    auto go = [&](auto prec) -> hipError_t {
        using T = decltype(prec);
        AkBatch<T> b{};
        for (int j = 0; j < count; ++j) {
            b.lk[j] = record_at<T>(e, e.ak_rec[j]).fib;
            b.ws[j] = e.ak_ws[j];
        }
        b.count = count;
        hipLaunchKernelGGL((k_link_sums<T>), dim3(nb), dim3(BX), 0, e.stream, e.ak_buf,
                           e.two_node ? (const double*)e.tq_buf : nullptr, b, lgr,
                           (uint32_t)e.n_links);
        return hipGetLastError();
    };
    return e.precision == 1 ? go(float{}) : go(double{});
}

hipError_t launch_link_gradients(Engine& e, double* dq, double* dphi) {
    if (!e.n_links || (!dq && !dphi)) return hipSuccess;
    auto go = [&](auto lat) {
        using L = decltype(lat);
        hipLaunchKernelGGL((k_link_finish<L>), dim3((unsigned)((e.n_links + BX - 1) / BX)),
                           dim3(BX), 0, e.stream, e.d_gq, e.d_gs, e.d_lkderiv, e.d_lkc4,
                           e.d_lkdir, e.d_perm, e.rho0, (uint32_t)e.n_links, dq, dphi);
        return hipGetLastError();
    };
    if (e.lattice == 0) return go(D2Q9{});
    if (e.lattice == 2) return go(D3Q15{});
    return go(D3Q19{});
}

hipError_t launch_two_node_adjoint(Engine& e, const Snapshot* next, const void* fib_next,
                                   void* lam_in, const AdjointObjective& obj) {
    if (e.n_links == 0) return hipSuccess;
    const Grid g = adj_grid(e);
    AdjArgs a;
    a.obj_kind = obj.kind;
    a.obj_tag = obj.tag;
    a.w_force = obj.kind == 1 ? obj.weight : 0.0;
    a.w_ux = 0.0;
    a.want_ds = 0;
    a.x_in = a.x_out = 0u;
    a.a_in = a.a_out = 0.0;
    const unsigned nb = (unsigned)((e.n_links + BX - 1) / BX);
    // on records (fib_next given) the term goes into the step's run of
    // tq_buf, the run the following launch_adjoint_step fills in ak_buf
    const bool store = fib_next != nullptr;
    if (store && !e.tq_buf) return hipErrorInvalidValue;
    if (store && e.ak_pending == kAkBatch) {
        const hipError_t fs = launch_link_sums(e);
        if (fs != hipSuccess) return fs;
    }
    double* gq = store ? e.tq_buf + (size_t)e.ak_pending * (size_t)std::max<int64_t>(e.n_links, 1)
                       : e.d_gq;
    return adj_dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_two_node_pre<L, T, XB>), dim3(nb), dim3(BX), 0, e.stream,
                           next ? (const T*)next->f : nullptr, (const T*)fib_next,
                           (T*)lam_in, e.d_lknode, e.d_lkdir, e.d_lktag,
                           e.d_lkc1d, e.d_lkd1d, gq, store ? 1 : 0, (uint32_t)e.n_links, g,
                           adj_params<L, T>(e), a);
        return hipGetLastError();
    });
}

hipError_t launch_link_pull(Engine& e, const Snapshot& s, void* out) {
    if (e.n_links == 0) return hipSuccess;
    const Grid g = adj_grid(e);
    const unsigned nb = (unsigned)((e.n_links + BX - 1) / BX);
    return adj_dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_link_pull<L, T, XB>), dim3(nb), dim3(BX), 0, e.stream,
                           (const T*)s.f, e.d_lknode, e.d_lkdir, (uint32_t)e.n_links, g,
                           adj_params<L, T>(e), (T*)out);
        return hipGetLastError();
    });
}

hipError_t launch_adjoint_out(Engine& e, const void* lam, double* out) {
    const unsigned nb = (unsigned)((e.N + BX - 1) / BX);
    return adj_dispatch(e, [&](auto lat, auto prec, auto) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        hipLaunchKernelGGL((k_adjoint_out<L, T>), dim3(nb), dim3(BX), 0, e.stream,
                           (const T*)lam, e.d_info, (uint32_t)e.N, out);
        return hipGetLastError();
    });
}

}  // namespace lbe
