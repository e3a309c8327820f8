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
__device__ __forceinline__ void block_accumulate(double (&v)[NC], double* __restrict__ dst) {
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

template <class L, class T, int XB>
__global__ void __launch_bounds__(BX)
k_adjoint(const T* __restrict__ A, const T* __restrict__ wa,
          const T* __restrict__ lam_in, T* __restrict__ lam_out,
          const int32_t* __restrict__ nodeword, const uint8_t* __restrict__ lkdir,
          const LinkCoef* __restrict__ lkcoef, const LinkDeriv* __restrict__ lkderiv,
          const double* __restrict__ lkc4, const int32_t* __restrict__ lktag,
          double* __restrict__ gq, double* __restrict__ gphi,
          double* __restrict__ gglob, Grid g, Params<L, T> p, AdjArgs a) {
    constexpr int Q = L::Q, D = L::D;
    constexpr int NC = D + Q;
    const NodePos pos = node_of_thread(g);
    const int32_t nw = pos.in ? nodeword[pos.n] : -1;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;

    if (nw >= 0) {
        const NodeLinks nl = node_links(nw, lkdir);
        // forward recomputation at this node
        T f0[Q];
        pull<L, T, XB>(A, wa, g, pos, p, nl, f0);
        const Macro<L, T> mac = moments<L, T>(f0, p.inv_rho0);
        T mneq[Q];
        {
            T d[Q];
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                d[i] = f0[i] - feq<L, T, i>(mac, p.rho0);
            });
            unroll<Q>([&](auto K) {
                constexpr int k = decltype(K)::value;
                T s = 0;
                if constexpr (!L::conserved(k))
                    unroll<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        macc<TAB<L>.M[k][i]>(s, d[i]);
                    });
                mneq[k] = s;
            });
        }
        T fp[Q];
        unroll<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            T s = 0;
            unroll<Q>([&](auto K) {
                constexpr int k = decltype(K)::value;
                if constexpr (!L::conserved(k)) macc<TAB<L>.M[k][i]>(s, mneq[k] * p.rate[k]);
            });
            fp[i] = f0[i] - s + p.force[i];
        });

        // mu: adjoint of the post-collision values at this node
        T mu[Q];
        T dir[Q];
        const Push<XB> ps(g, pos);
        unroll<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int ib = TAB<L>.opp[i];
            dir[i] = 0;
            mu[i] = 0;
            if constexpr (i == 0) {
                mu[i] = lam_in[pos.n];
            } else {
                const bool into_wall = (nl.mask >> ib) & 1u;
                bool lost = into_wall;
                if constexpr (XB == XBC_OUTFLOW && L::E[i][0] == 1) lost = lost || ps.x_out;
                if (!lost) mu[i] = lam_in[(size_t)i * g.N + ps.template dst<L, i>()];
                if constexpr (XB == XBC_OUTFLOW && L::E[i][0] == -1) {
                    if (ps.x_out) {
                        const uint32_t n2 = ps.template dst_clamped<L, i>(pos.ix);
                        if (nodeword[n2] >= 0) mu[i] += lam_in[(size_t)i * g.N + n2];
                    }
                }
            }
        });

        // own cut links: Eq. (213) reversed, objective terms, per-link gradients
        if (nl.mask) {
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int ib = TAB<L>.opp[i];
                if constexpr (i > 0) {
                    if ((nl.mask >> i) & 1u) {
                        const uint32_t k = link_index(nl, i);
                        double ak = (double)lam_in[(size_t)i * g.N + pos.n];
                        if (a.obj_kind == 1 && lktag[k] == a.obj_tag && L::E[i][0] != 0) {
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
                        gq[k] += ak * (dc.d1 * (double)f0[ib] + dc.d2 * (double)fp[i] +
                                       dc.d3 * (double)fp[ib] + dc.dwall);
                        const double c4w = lkc4[k] * 3.0 * L::W[i] * p.rho0_d * ak;
#pragma unroll
                        for (int al = 0; al < D; ++al)
                            gphi[(size_t)k * D + al] += c4w * L::E[i][al];
                    }
                }
            });
        }

        // dJ/dg and dJ/ds partials
        unroll<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double m3 = 3.0 * L::W[i] * p.rho0_d * (double)mu[i];
#pragma unroll
            for (int al = 0; al < D; ++al)
                if (L::E[i][al] != 0) acc[al] += L::E[i][al] * m3;
        });

        // collision adjoint
        T qm[Q];
        unroll<Q>([&](auto K) {
            constexpr int k = decltype(K)::value;
            T s = 0;
            if constexpr (!L::conserved(k))
                unroll<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    macc<TAB<L>.M[k][i]>(s, mu[i]);
                });
            qm[k] = s;
        });
        if (a.want_ds) {
            unroll<Q>([&](auto K) {
                constexpr int k = decltype(K)::value;
                if constexpr (!L::conserved(k))
                    acc[D + k] -= (double)qm[k] * (double)mneq[k] / (double)TAB<L>.norm[k];
            });
        }
        T v[Q];
        unroll<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            T s = 0;
            unroll<Q>([&](auto K) {
                constexpr int k = decltype(K)::value;
                if constexpr (!L::conserved(k)) macc<TAB<L>.M[k][i]>(s, qm[k] * p.rate[k]);
            });
            v[i] = s;
        });
        // J^T v = a_s + b.e_j
        T as = 0, bx = 0, by = 0, bz = 0;
        unroll<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const T wv = T(L::W[i]) * v[i];
            as += wv;
            T eu = 0;
            macc<L::E[i][0]>(eu, mac.u[0]);
            macc<L::E[i][1]>(eu, mac.u[1]);
            macc<L::E[i][2]>(eu, mac.u[2]);
            const T c = T(3) + T(9) * eu;
            macc<L::E[i][0]>(bx, c * wv);
            macc<L::E[i][1]>(by, c * wv);
            macc<L::E[i][2]>(bz, c * wv);
        });
        bx -= T(3) * mac.u[0] * as;
        by -= T(3) * mac.u[1] * as;
        bz -= T(3) * mac.u[2] * as;
        const T wux = (T)a.w_ux;
        unroll<Q>([&](auto J) {
            constexpr int j = decltype(J)::value;
            T jt = as;
            macc<L::E[j][0]>(jt, bx);
            macc<L::E[j][1]>(jt, by);
            macc<L::E[j][2]>(jt, bz);
            T out = mu[j] - v[j] + jt + dir[j];
            if (a.obj_kind == 2) macc<L::E[j][0]>(out, wux);
            lam_out[(size_t)j * g.N + pos.n] = out;
        });
    }

    // b is uniform over the block, so the barrier inside is block-uniform
    uint32_t b = blockIdx.x;
    if (g.chunk) b = (b % NXCD) * g.chunk + b / NXCD;
    if (b < g.nblocks) block_accumulate<NC>(acc, gglob + (size_t)b * NC);
}

template <class L, class T>
__global__ void __launch_bounds__(BX)
k_adjoint_out(const T* __restrict__ lam, const int32_t* __restrict__ nodeword,
              uint32_t N, double* __restrict__ out) {
    const uint32_t n = blockIdx.x * BX + threadIdx.x;
    if (n >= N) return;
    const bool fluid = nodeword[n] >= 0;
    for (int i = 0; i < L::Q; ++i)
        out[(size_t)i * N + n] = fluid ? (double)lam[(size_t)i * N + n] : 0.0;
}

// ----------------------------------------------------------------------------

template <class L, class T>
static Params<L, T> adj_params(const Engine& e) {
    Params<L, T> p;
    for (int k = 0; k < L::Q; ++k)
        p.rate[k] = (T)(L::conserved(k) ? 0.0 : e.s[k] / (double)TAB<L>.norm[k]);
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
    return p;
}

static Grid adj_grid(const Engine& e) {
    Grid g;
    g.nx = (uint32_t)e.nx;
    g.ny = (uint32_t)e.ny;
    g.nz = (uint32_t)e.nz;
    g.N = (uint32_t)e.N;
    g.bpr = (uint32_t)((e.nx + BX - 1) / BX);
    g.nblocks = g.bpr * g.ny * g.nz;
    g.chunk = (g.nblocks + NXCD - 1) / NXCD;
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
    a.want_ds = 1;
    return adj_dispatch(e, [&](auto lat, auto prec, auto xb) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        constexpr int XB = decltype(xb)::value;
        hipLaunchKernelGGL((k_adjoint<L, T, XB>), dim3(g.chunk * NXCD), dim3(BX), 0,
                           e.stream, (const T*)fwd.f, (const T*)fwd.wa,
                           (const T*)lam_in, (T*)lam_out, e.d_nodeword, e.d_lkdir,
                           e.d_lkcoef, e.d_lkderiv, e.d_lkc4, e.d_lktag, e.d_gq,
                           e.d_gphi, e.d_gglob, g, adj_params<L, T>(e), a);
        return hipGetLastError();
    });
}

hipError_t launch_adjoint_out(Engine& e, const void* lam, double* out) {
    const unsigned nb = (unsigned)((e.N + BX - 1) / BX);
    return adj_dispatch(e, [&](auto lat, auto prec, auto) -> hipError_t {
        using L = decltype(lat);
        using T = decltype(prec);
        hipLaunchKernelGGL((k_adjoint_out<L, T>), dim3(nb), dim3(BX), 0, e.stream,
                           (const T*)lam, e.d_nodeword, (uint32_t)e.N, out);
        return hipGetLastError();
    });
}

}  // namespace lbe
