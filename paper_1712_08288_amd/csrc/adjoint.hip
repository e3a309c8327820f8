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
// Gradients accumulated on the way, in double:
//   dJ/dgamma_k += a_k (dc1 f_ibar + dc2 g_i + dc3 g_ibar + dwall),
//   dJ/dphi_k   += a_k c4 3 w_i rho0 e_i,
//   dJ/dg       += sum_i mu_i 3 w_i rho0 e_i,
//   dJ/ds_k     += -(M mu)_k (M (f - f^eq))_k / |M_k|^2,
// where a_k is the adjoint of the link value f_i(y, t+1).
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
};

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

// Lattice data of a direction known only at run time (link lanes).
template <class L>
__device__ __forceinline__ void dir_data(int d, int (&e)[3], double& w) {
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (i == d) {
            e[0] = L::E[i][0];
            e[1] = L::E[i][1];
            e[2] = L::E[i][2];
            w = L::W[i];
        }
    });
}

// Link k = (y, i) of a mixed wave, handled by the lane of its node y: the
// contribution of its adjoint a_k to mu and to lambda(y, t), and its
// gradients.  Used for links past the 64th of a wave (the first 64 go
// through the wave's LDS slab).
template <class L, class T, int i>
__device__ __forceinline__ void own_link_direct(uint32_t k, const T* __restrict__ lam_in,
                                                uint32_t n, uint32_t S,
                                                const LinkCoef* __restrict__ lkcoef,
                                                const LinkDeriv* __restrict__ lkderiv,
                                                const double* __restrict__ lkc4,
                                                const int32_t* __restrict__ lktag,
                                                double* __restrict__ gq, double* __restrict__ gphi,
                                                const Params<L, T>& p, const AdjArgs& a,
                                                const T (&f)[L::Q], const T (&fp)[L::Q],
                                                T (&mu)[L::Q], T (&dir)[L::Q]) {
    constexpr int ib = TAB<L>.opp[i];
    double ak = (double)ld(lam_in + (size_t)i * S, n);
    if (a.obj_kind == 1 && L::E[i][0] != 0 && lktag[k] == a.obj_tag) {
        // drag: (e_ibar)_x (f'_ibar(y,t) + f_i(y,t+1))
        const double dfx = -(double)L::E[i][0] * a.w_force;
        ak += dfx;
        mu[ib] += (T)dfx;
    }
    const LinkCoef c = lkcoef[k];
    const LinkDeriv dc = lkderiv[k];
    mu[i] += (T)(c.c2 * ak);
    mu[ib] += (T)(c.c3 * ak);
    dir[i] += (T)(p.c0 * ak);
    dir[ib] += (T)(c.c1 * ak);
    gq[k] += ak * (dc.d1 * (double)f[ib] + dc.d2 * (double)fp[i] + dc.d3 * (double)fp[ib] +
                   p.wall_scale * dc.dwall);
    const double c4w = lkc4[k] * 3.0 * L::W[i] * p.rho0_d * p.wall_scale * ak;
#pragma unroll
    for (int al = 0; al < L::D; ++al)
        if (L::E[i][al] != 0) gphi[(size_t)k * L::D + al] += c4w * L::E[i][al];
}

// Mixed waves handle their cut links cooperatively (see LinkStage): the
// link lanes read the link data and a_k = lambda_i(y, t+1) (plus the drag
// term) with coalesced loads and hand c2 a_k, c3 a_k (+ drag), c0 a_k and
// c1 a_k to the node's lane through LDS; the node's lane hands back
// f_ibar(y,t), f'_i(y,t) and f'_ibar(y,t) for the link lanes' gradients.
template <class L, class T, int XB, bool WANT_DS, bool ROWS>
__global__ void __launch_bounds__(BX)
k_adjoint(const T* __restrict__ A, const T* __restrict__ wa,
          const T* __restrict__ lam_in, T* __restrict__ lam_out,
          NodeMeta nm, const LinkCoef* __restrict__ lkcoef,
          const LinkDeriv* __restrict__ lkderiv,
          const double* __restrict__ lkc4, const int32_t* __restrict__ lktag,
          const uint8_t* __restrict__ lkdir, const int32_t* __restrict__ lknode,
          double* __restrict__ gq, double* __restrict__ gphi,
          double* __restrict__ gglob, Grid g, Params<L, T> p, AdjArgs a) {
    constexpr int Q = L::Q, D = L::D, NP = NPAIR<L>;
    constexpr int NC = D + Q;                 // layout of the per-block sums
    constexpr int NR = WANT_DS ? NC : D;      // columns reduced here
    __shared__ LinkStage<T> stage[BX / 64];
    const NodePos pos = node_of_thread<ROWS>(g);
    uint32_t lb = blockIdx.x;
    if (g.chunk) lb = (lb % NXCD) * g.chunk + lb / NXCD;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint2 wv = lb < g.nblocks ? nm.wave[lb * (BX / 64) + wid] : uint2{WAVE_IDLE, 0u};
    const uint32_t kind = wave_kind(wv);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nlw = wave_links(wv), wbase = wv.y;
    LinkStage<T>& st = stage[wid];
    double acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] = 0.0;

    // loads that do not depend on the node's metadata are issued first:
    // the planes of the forward pull and the adjoint gathers
    // lambda_i(y + e_i, t+1) (entries of solid or absent neighbours are
    // read and then discarded)
    T f[Q], lg[Q];
    const Push<XB> ps(g, pos);
    if (kind != WAVE_IDLE && pos.in) {
        pull_planes<L, T, XB>(A, g, pos, p, NodeLinks{0u, 0u}, f);
        unroll<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            lg[i] = ld(lam_in + (size_t)i * g.S, i == 0 ? pos.n : ps.template dst<L, i>());
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
        // forward state f(y, t) and its velocity
        T sp[NP], dp[NP];
        pair_split<L, T>(f, sp, dp);
        T rho, j[3];
        conserved_of<L, T>(f[0], sp, dp, rho, j);
        const T u[3] = {j[0] * p.inv_rho0, j[1] * p.inv_rho0, j[2] * p.inv_rho0};

        // mu_i(y) = dJ/df'_i(y): lambda_i(y + e_i, t+1) where that node pulls
        T mu[Q], dir[Q];
        unroll<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int ib = TAB<L>.opp[i];
            dir[i] = 0;
            if constexpr (i == 0) {
                mu[i] = lg[0];
            } else {
                bool lost = (nl.mask >> ib) & 1u;     // y + e_i is solid
                if constexpr (XB == XBC_OUTFLOW && L::E[i][0] == 1) lost = lost || ps.x_out;
                mu[i] = lost ? T(0) : lg[i];
                if constexpr (XB == XBC_OUTFLOW && L::E[i][0] == -1) {
                    if (ps.x_out) {
                        const uint32_t n2 = ps.template dst_clamped<L, i>(pos.ix);
                        if (!is_solid(nm.info[n2])) mu[i] += ld(lam_in + (size_t)i * g.S, n2);
                    }
                }
            }
        });

        // own cut links: Eq. (213) reversed, drag terms, per-link gradients
        if (!PLAIN && nl.mask) {
            T fp[Q];
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                fp[i] = f[i];
            });
            Macro<L, T> mac;
            collide<L, T>(fp, p, mac);
            uint32_t k = nl.base;
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int ib = TAB<L>.opp[i];
                if constexpr (i > 0) {
                    const uint32_t bit = (nl.mask >> i) & 1u;
                    if (bit) {
                        if (k < 64u) {
                            mu[i] += st.v[0][k];
                            mu[ib] += st.v[1][k];
                            dir[i] += st.v[2][k];
                            dir[ib] += st.v[3][k];
                            st.v[0][k] = f[ib];
                            st.v[1][k] = fp[i];
                            st.v[2][k] = fp[ib];
                        } else {
                            own_link_direct<L, T, i>(wbase + k, lam_in, pos.n, g.S, lkcoef,
                                                     lkderiv, lkc4, lktag, gq, gphi, p, a, f,
                                                     fp, mu, dir);
                        }
                    }
                    k += bit;
                }
            });
        }

        // collision adjoint: lambda = mu - v + J^T v, v = M^T R M mu
        T smu[NP], dmu[NP];
        pair_split<L, T>(mu, smu, dmu);
        T qm[Q];
        moments_of<L, T>(mu[0], smu, dmu, qm);
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
        auto finish = [&](auto J, T v) {
            constexpr int jd = decltype(J)::value;
            T out = mu[jd] - v + as + dir[jd];
            macc<L::E[jd][0]>(out, b[0]);
            macc<L::E[jd][1]>(out, b[1]);
            macc<L::E[jd][2]>(out, b[2]);
            if (a.obj_kind == 2) macc<L::E[jd][0]>(out, wux);
            st_nt(lam_out + (size_t)jd * g.S, pos.n, out);
        };
        finish(std::integral_constant<int, 0>{}, e0);
        unroll<NP>([&](auto P) {
            constexpr int pp = decltype(P)::value;
            constexpr int i = DER<L>.pi[pp];
            constexpr int ib = TAB<L>.opp[i];
            finish(std::integral_constant<int, i>{}, ev[pp] + od[pp]);
            finish(std::integral_constant<int, ib>{}, ev[pp] - od[pp]);
        });

        // dJ/dg += 3 rho0 sum_i w_i e_i mu_i (pair form: w_i e_i (mu_i - mu_ibar)),
        // summed over the node in T, accumulated over nodes in double
        T sg[3] = {0, 0, 0};
        unroll<NP>([&](auto P) {
            constexpr int pp = decltype(P)::value;
            constexpr int i = DER<L>.pi[pp];
            const T t = T(L::W[i]) * dmu[pp];
            macc<L::E[i][0]>(sg[0], t);
            macc<L::E[i][1]>(sg[1], t);
            macc<L::E[i][2]>(sg[2], t);
        });
#pragma unroll
        for (int al = 0; al < D; ++al) acc[al] += 3.0 * p.rho0_d * (double)sg[al];
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

    if (kind == WAVE_PLAIN) {
        node(std::true_type{}, NodeLinks{0u, 0u});
    } else if (kind == WAVE_MIXED) {
        const uint32_t info = pos.in ? nm.info[pos.n] : kInfoSolid;
        const bool sol = is_solid(info);
        const NodeLinks nl = sol ? NodeLinks{0u, 0u} : node_links(info, 0u);
        // forward state: the link slots of the recorded step
        const T wa0 = lane < nlw ? wa[wbase + lane] : T(0);
        wave_link_values<L, T>(wa, wbase, lane, wa0, nl, st, f);
        if (p.c1d) complete_two_node<L, T>(p.c1d + wbase, nl, f);
        // link lanes: a_k and the pieces of mu and lambda(y, t) it feeds
        double ak = 0.0;
        int ld_dir = 0;
        if (lane < nlw && lane < 64u) {
            const uint32_t k = wbase + lane;
            ld_dir = lkdir[k];
            int e[3];
            double w;
            dir_data<L>(ld_dir, e, w);
            ak = (double)lam_in[(size_t)ld_dir * g.S + (uint32_t)lknode[k]];
            double dfx = 0.0;
            if (a.obj_kind == 1 && e[0] != 0 && lktag[k] == a.obj_tag) {
                // drag: (e_ibar)_x (f'_ibar(y,t) + f_i(y,t+1))
                dfx = -(double)e[0] * a.w_force;
                ak += dfx;
            }
            const LinkCoef c = lkcoef[k];
            st.v[0][lane] = (T)(c.c2 * ak);
            st.v[1][lane] = (T)(c.c3 * ak + dfx);
            st.v[2][lane] = (T)(p.c0 * ak);
            st.v[3][lane] = (T)(c.c1 * ak);
        }
        wave_lds_sync();
        if (!sol) node(std::false_type{}, nl);
        wave_lds_sync();
        // link lanes: per-link gradients from the node's values
        if (lane < nlw && lane < 64u) {
            const uint32_t k = wbase + lane;
            const LinkDeriv dc = lkderiv[k];
            gq[k] += ak * (dc.d1 * (double)st.v[0][lane] + dc.d2 * (double)st.v[1][lane] +
                           dc.d3 * (double)st.v[2][lane] + p.wall_scale * dc.dwall);
            int e[3];
            double w;
            dir_data<L>(ld_dir, e, w);
            const double c4w = lkc4[k] * 3.0 * w * p.rho0_d * p.wall_scale * ak;
#pragma unroll
            for (int al = 0; al < D; ++al)
                if (e[al] != 0) gphi[(size_t)k * D + al] += c4w * e[al];
        }
        // the solid lanes store NaN (nothing reads lambda at solid nodes) so
        // that the wave writes whole lines of lam_out: partial lines cost
        // HBM read-modify-write cycles
        if (pos.in && sol) {
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                st_nt(lam_out + (size_t)i * g.S, pos.n, (T)__builtin_nan(""));
            });
        }
    }

    // lb is uniform over the block, so the barrier inside is block-uniform
    if (lb < g.nblocks) block_accumulate<NR>(acc, gglob + (size_t)lb * NC);
}

// Eq. (211) links k = (x_f, i) with a deferred c1: the link value is
// f_i(x_f, t+1) = (terms at t) + c1 f_ibar(x_f, t+1), so its adjoint a_k also
// reaches f_ibar(x_f, t+1) (whose own adjoint the node x_f + e_i gathers in
// the next kernel) and dJ/dgamma gets a_k dc1 f_ibar(x_f, t+1).
template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_two_node_pre(const T* __restrict__ A_next, T* __restrict__ lam_in,
               const int32_t* __restrict__ lknode, const uint8_t* __restrict__ lkdir,
               const int32_t* __restrict__ lktag, const double* __restrict__ c1d,
               const double* __restrict__ d1d, double* __restrict__ gq,
               uint32_t n_links, Grid g, Params<L, T> p, AdjArgs a) {
    const uint32_t k = blockIdx.x * BX + threadIdx.x;
    if (k >= n_links) return;
    const double c = c1d[k];
    if (c == 0.0) return;
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
    double ak = (double)lam_in[(size_t)i * g.S + n];
    if (a.obj_kind == 1 && ex != 0 && lktag[k] == a.obj_tag) ak += -(double)ex * a.w_force;
    T* dst = lam_in + (size_t)ib * g.S + n;
    *dst = (T)((double)*dst + c * ak);
    gq[k] += ak * d1d[k] * (double)pull_one<L, T, XB>(A_next, g, p, n, ib);
}

template <class L, class T>
__global__ void __launch_bounds__(BX)
k_adjoint_out(const T* __restrict__ lam, const uint32_t* __restrict__ info,
              uint32_t N, uint32_t S, double* __restrict__ out) {
    const uint32_t n = blockIdx.x * BX + threadIdx.x;
    if (n >= N) return;
    const bool fluid = !is_solid(info[n]);
    for (int i = 0; i < L::Q; ++i)
        out[(size_t)i * N + n] = fluid ? (double)lam[(size_t)i * S + n] : 0.0;
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
    g.nblocks = (uint32_t)((e.N + BX - 1) / BX);
    g.bpr = e.nx % BX == 0 ? (uint32_t)(e.nx / BX) : 0u;
    g.chunk = e.xcd_remap ? (g.nblocks + NXCD - 1) / NXCD : 0;
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

hipError_t launch_adjoint_step(Engine& e, const Snapshot& fwd, const void* lam_in,
                               void* lam_out, const AdjointObjective& obj) {
    const Grid g = adj_grid(e);
    AdjArgs a;
    a.obj_kind = obj.kind;
    a.obj_tag = obj.tag;
    a.w_force = obj.kind == 1 ? obj.weight : 0.0;
    a.w_ux = obj.kind == 2 ? obj.weight * obj.inv_nfluid / e.rho0 : 0.0;
    a.want_ds = e.want_ds ? 1 : 0;
    return adj_dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        auto kern = a.want_ds ? (g.bpr ? k_adjoint<L, T, XB, true, true> : k_adjoint<L, T, XB, true, false>)
                              : (g.bpr ? k_adjoint<L, T, XB, false, true> : k_adjoint<L, T, XB, false, false>);
        hipLaunchKernelGGL(kern, dim3(g.chunk ? g.chunk * NXCD : g.nblocks), dim3(BX), 0,
                           e.stream, (const T*)fwd.f, (const T*)fwd.wa,
                           (const T*)lam_in, (T*)lam_out,
                           NodeMeta{e.d_info, e.d_wave}, e.d_lkcoef, e.d_lkderiv, e.d_lkc4, e.d_lktag,
                           e.d_lkdir, e.d_lknode, e.d_gq,
                           e.d_gphi, e.d_gglob, g, adj_params<L, T>(e), a);
        return hipGetLastError();
    });
}

hipError_t launch_two_node_adjoint(Engine& e, const Snapshot& next, void* lam_in,
                                   const AdjointObjective& obj) {
    if (e.n_links == 0) return hipSuccess;
    const Grid g = adj_grid(e);
    AdjArgs a;
    a.obj_kind = obj.kind;
    a.obj_tag = obj.tag;
    a.w_force = obj.kind == 1 ? obj.weight : 0.0;
    a.w_ux = 0.0;
    a.want_ds = 0;
    const unsigned nb = (unsigned)((e.n_links + BX - 1) / BX);
    return adj_dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_two_node_pre<L, T, XB>), dim3(nb), dim3(BX), 0, e.stream,
                           (const T*)next.f, (T*)lam_in, e.d_lknode, e.d_lkdir, e.d_lktag,
                           e.d_lkc1d, e.d_lkd1d, e.d_gq, (uint32_t)e.n_links, g,
                           adj_params<L, T>(e), a);
        return hipGetLastError();
    });
}

hipError_t launch_adjoint_out(Engine& e, const void* lam, double* out) {
    const unsigned nb = (unsigned)((e.N + BX - 1) / BX);
    return adj_dispatch(e, [&](auto lat, auto prec, auto) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        hipLaunchKernelGGL((k_adjoint_out<L, T>), dim3(nb), dim3(BX), 0, e.stream,
                           (const T*)lam, e.d_info, (uint32_t)e.N, (uint32_t)e.S, out);
        return hipGetLastError();
    });
}

}  // namespace lbe
