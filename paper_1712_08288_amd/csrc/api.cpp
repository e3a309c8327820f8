// C ABI of the engine: validation, per-link coefficient set-up in double,
// device memory, the time loop, checkpointed runs and the reverse sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "engine.hpp"
#include "geometry.hpp"
#include "lattice.hpp"

using lbe::Engine;
using lbe::Snapshot;

struct lbm {
    Engine e;
};

namespace {

int fail(lbm_t* h, int code, const std::string& msg) {
    if (h) h->e.err = msg;
    return code;
}

#define HIPCHK(h, call)                                                              \
    do {                                                                             \
        hipError_t _st = (call);                                                     \
        if (_st != hipSuccess)                                                       \
            return fail((h), LBM_EDEVICE,                                            \
                        std::string(#call) + ": " + hipGetErrorString(_st));         \
    } while (0)

// ---- lattice tables on the host (the same constexpr definitions) -------------
// host-side lattice data by runtime id (LBM_D2Q9, LBM_D3Q19, LBM_D3Q15)
template <class F>
auto with_lattice(int lattice, F&& f) {
    if (lattice == LBM_D2Q9) return f(lbe::D2Q9{});
    if (lattice == LBM_D3Q15) return f(lbe::D3Q15{});
    return f(lbe::D3Q19{});
}
int lat_Q(int lattice) {
    return with_lattice(lattice, [](auto l) { return decltype(l)::Q; });
}
int lat_D(int lattice) {
    return with_lattice(lattice, [](auto l) { return decltype(l)::D; });
}
int lat_e(int lattice, int i, int a) {
    return with_lattice(lattice, [&](auto l) { return decltype(l)::E[i][a]; });
}
double lat_w(int lattice, int i) {
    return with_lattice(lattice, [&](auto l) { return decltype(l)::W[i]; });
}
int lat_M(int lattice, int k, int i) {
    return with_lattice(lattice, [&](auto l) { return lbe::TAB<decltype(l)>.M[k][i]; });
}
bool lat_conserved(int lattice, int k) {
    return with_lattice(lattice, [&](auto l) { return decltype(l)::conserved(k); });
}

// ---- the free parameter l(gamma) (paper, Section 3 and Eq. (212)) ------------
double l_of(int rule, double g) {
    switch (rule) {
        case LBM_L_GAMMA: return g;
        case LBM_L_1P5GAMMA: return 1.5 * g;
        case LBM_L_2GAMMA: return 2.0 * g;
        case LBM_L_GAMMA2: return g * g;
        case LBM_L_GAMMA2_PLUS_GAMMA: return g * g + g;
        case LBM_L_ZERO: return 0.0;
        default: return 2.0 * g - 1.0 > 0.0 ? 2.0 * g - 1.0 : 0.0;
    }
}
double dl_of(int rule, double g) {
    switch (rule) {
        case LBM_L_GAMMA: return 1.0;
        case LBM_L_1P5GAMMA: return 1.5;
        case LBM_L_2GAMMA: return 2.0;
        case LBM_L_GAMMA2: return 2.0 * g;
        case LBM_L_GAMMA2_PLUS_GAMMA: return 2.0 * g + 1.0;
        case LBM_L_ZERO: return 0.0;
        default: return 2.0 * g - 1.0 > 0.0 ? 2.0 : 0.0;
    }
}

template <class T>
void free_dev(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void free_snap(Snapshot& s) {
    if (s.f) (void)hipFree(s.f);
    if (s.wa) (void)hipFree(s.wa);
    s.f = s.wa = nullptr;
}

size_t f_bytes(const Engine& e) { return (size_t)e.Q * (size_t)e.S * e.elem; }
size_t rec_bytes(const Engine& e) { return (size_t)lbe::record_values(e) * e.elem; }

// the reverse sweep can run on step records instead of the forward states
// (see Engine::rec_last): everything but the rate gradients
bool velocity_mode(const Engine& e) { return !e.want_ds; }

// the link run (f_ibar(x_f, t) of every link) of a step record
const void* record_links(const Engine& e, const void* rec) {
    return (const char*)rec + (size_t)e.D * (size_t)e.S * e.elem;
}

void free_list(std::vector<void*>& v) {
    for (auto& p : v)
        if (p) (void)hipFree(p);
    v.clear();
}

int alloc_list(lbm_t* h, std::vector<void*>& v, size_t count, size_t bytes) {
    if (v.size() == count) return LBM_OK;
    free_list(v);
    v.assign(count, nullptr);
    for (auto& p : v)
        if (hipMalloc(&p, bytes) != hipSuccess) {
            p = nullptr;
            free_list(v);
            return fail(h, LBM_ENOMEM, "device allocation of step records failed");
        }
    return LBM_OK;
}

// Nodes per array slot count: N rounded up to whole population blocks (the
// population arrays hold Q * S values in blocks of 2048 nodes; the velocity
// records hold D planes of stride S).
int64_t plane_stride(int64_t N) { return ((N + 2047) / 2048) * 2048; }
size_t wa_bytes(const Engine& e) {
    return (size_t)std::max<int64_t>(e.n_links, 1) * e.elem;
}

int alloc_snap(lbm_t* h, Snapshot& s) {
    Engine& e = h->e;
    if (hipMalloc(&s.f, f_bytes(e)) != hipSuccess) {
        s.f = nullptr;
        return fail(h, LBM_ENOMEM, "device allocation of a distribution array failed");
    }
    if (hipMalloc(&s.wa, wa_bytes(e)) != hipSuccess) {
        (void)hipFree(s.f);
        s.f = nullptr;
        s.wa = nullptr;
        return fail(h, LBM_ENOMEM, "device allocation of link slots failed");
    }
    return LBM_OK;
}

int copy_snap(lbm_t* h, const Snapshot& dst, const Snapshot& src) {
    Engine& e = h->e;
    HIPCHK(h, hipMemcpyAsync(dst.f, src.f, f_bytes(e), hipMemcpyDeviceToDevice, e.stream));
    HIPCHK(h, hipMemcpyAsync(dst.wa, src.wa, wa_bytes(e), hipMemcpyDeviceToDevice, e.stream));
    return LBM_OK;
}

int ensure_scratch(lbm_t* h, int64_t n_doubles) {
    Engine& e = h->e;
    if (e.scratch_len >= n_doubles) return LBM_OK;
    free_dev(e.d_scratch);
    if (hipMalloc((void**)&e.d_scratch, (size_t)n_doubles * sizeof(double)) != hipSuccess) {
        e.d_scratch = nullptr;
        e.scratch_len = 0;
        return fail(h, LBM_ENOMEM, "device scratch allocation failed");
    }
    e.scratch_len = n_doubles;
    return LBM_OK;
}

template <class T>
int upload(lbm_t* h, T*& dst, const T* src, size_t n) {
    free_dev(dst);
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (hipMalloc((void**)&dst, bytes) != hipSuccess) {
        dst = nullptr;
        return fail(h, LBM_ENOMEM, "device allocation failed");
    }
    if (n) HIPCHK(h, hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, h->e.stream));
    return LBM_OK;
}

int sync(lbm_t* h) {
    HIPCHK(h, hipStreamSynchronize(h->e.stream));
    return LBM_OK;
}

// Coefficients of Eq. (213) for every (sorted) link, and their gamma
// derivatives along l = l(gamma).
int compute_coefficients(lbm_t* h, std::vector<lbe::LinkCoef>& coef,
                         std::vector<lbe::LinkDeriv>& der, std::vector<double>& c4v,
                         std::vector<double>& c1d, std::vector<double>& d1d) {
    Engine& e = h->e;
    const int64_t L = e.n_links;
    coef.resize(L);
    der.resize(L);
    c4v.resize(L);
    c1d.resize(L);
    d1d.resize(L);
    const double b = e.b;
    for (int64_t k = 0; k < L; ++k) {
        const double g = e.q_h[k];
        const int i = e.lk_dir_h[k];
        const double l = l_of(e.l_rule, g);
        const double lp = dl_of(e.l_rule, g);
        const double lo = std::max(0.0, 2.0 * g - 1.0);
        if (!(l >= lo - 1e-12 && l <= 2.0 * g + 1e-12))
            return fail(h, LBM_EINVAL,
                        "l(gamma) outside the convex band max(0,2g-1) <= l <= 2g at link " +
                            std::to_string(e.perm[k]) + " (gamma = " + std::to_string(g) + ")");
        const double den = 1.0 + l;
        const double c1 = b * (1.0 + l - 2.0 * g) / den;
        const double c2 = b * l / den;
        const double c3 = b * (2.0 * g - l) / den;
        const double c4 = b * 2.0 / den;
        double ephi = 0.0;
        for (int a = 0; a < e.D; ++a) ephi += lat_e(e.lattice, i, a) * e.wall_u_h[k * e.D + a];
        const double unit = 3.0 * lat_w(e.lattice, i) * e.rho0 * ephi;
        const double den2 = den * den;
        const double d1 = b * ((lp - 2.0) * den - (1.0 + l - 2.0 * g) * lp) / den2;
        const double d2 = b * lp / den2;
        const double d3 = b * ((2.0 - lp) * den - (2.0 * g - l) * lp) / den2;
        const double d4 = -2.0 * b * lp / den2;
        // Eq. (211): the c1 term multiplies f_ibar(x_f, t+1) = f'_ibar(x_f + e_i, t)
        // and is added at the next pull, unless x_f + e_i is solid
        const bool defer = e.two_node && !e.ibar_is_link[k];
        coef[k] = {defer ? 0.0 : c1, c2, c3, c4 * unit};
        der[k] = {defer ? 0.0 : d1, d2, d3, d4 * unit};
        c1d[k] = defer ? c1 : 0.0;
        d1d[k] = defer ? d1 : 0.0;
        c4v[k] = c4;
    }
    return LBM_OK;
}

int upload_coefficients(lbm_t* h) {
    Engine& e = h->e;
    std::vector<lbe::LinkCoef> coef;
    std::vector<lbe::LinkDeriv> der;
    std::vector<double> c4v, c1d, d1d;
    int rc = compute_coefficients(h, coef, der, c4v, c1d, d1d);
    if (rc) return rc;
    if (e.precision == LBM_FP32) {
        std::vector<lbe::LinkCoefT<float>> cf(coef.size());
        for (size_t k = 0; k < coef.size(); ++k)
            cf[k] = {(float)coef[k].c1, (float)coef[k].c2, (float)coef[k].c3,
                     (float)coef[k].wall};
        // the upload is asynchronous: keep the host copy alive until the sync
        if ((rc = upload(h, e.d_lkcoef_f, cf.data(), cf.size()))) return rc;
        if ((rc = sync(h))) return rc;
    } else if ((rc = upload(h, e.d_lkcoef, coef.data(), coef.size()))) {
        return rc;
    }
    if ((rc = upload(h, e.d_lkderiv, der.data(), der.size()))) return rc;
    if ((rc = upload(h, e.d_lkc4, c4v.data(), c4v.size()))) return rc;
    if ((rc = upload(h, e.d_lkc1d, c1d.data(), c1d.size()))) return rc;
    if ((rc = upload(h, e.d_lkd1d, d1d.data(), d1d.size()))) return rc;
    return sync(h);
}

// Captured step loops become invalid when kernel arguments change.
void drop_graphs(Engine& e) {
    for (auto& g : e.graph_exec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Capture graph_steps consecutive steps starting from buffer `start` (an
// even count, so the graph starts and ends on the same buffer).
int build_graph(lbm_t* h, int start) {
    Engine& e = h->e;
    hipGraph_t graph = nullptr;
    HIPCHK(h, hipStreamBeginCapture(e.stream, hipStreamCaptureModeThreadLocal));
    int cur = start;
    hipError_t st = hipSuccess;
    for (int s = 0; s < e.graph_steps && st == hipSuccess; ++s) {
        st = lbe::launch_step(e, e.buf[cur], e.buf[cur ^ 1], lbe::StepObjective{});
        cur ^= 1;
    }
    const hipError_t st2 = hipStreamEndCapture(e.stream, &graph);
    if (st != hipSuccess || st2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(h, LBM_EDEVICE, std::string("graph capture: ") +
                                        hipGetErrorString(st != hipSuccess ? st : st2));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t st3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (st3 != hipSuccess)
        return fail(h, LBM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(st3));
    e.graph_exec[start] = exec;
    return LBM_OK;
}

void free_run(Engine& e) {
    for (auto& s : e.ckpt) free_snap(s);
    for (auto& s : e.pool) free_snap(s);
    e.ckpt.clear();
    e.pool.clear();
    free_list(e.rec_last);
    free_list(e.rec_pool);
    free_dev(e.fib_final);
    free_dev(e.fib_next);
    e.run_urec = false;
    for (auto& l : e.lam) {
        if (l) (void)hipFree(l);
        l = nullptr;
    }
    e.run_t0 = -1;
    e.run_n = 0;
    e.run_every = 0;
}

int zero(lbm_t* h, void* p, size_t bytes) {
    HIPCHK(h, hipMemsetAsync(p, 0, bytes, h->e.stream));
    return LBM_OK;
}

// one forward step from buf[cur] into buf[cur^1] (or between given
// snapshots), with the objective accumulated when `accumulate`; rec, when
// given, receives the step record (velocity of the state the step starts
// from, link values)
int forward_step(lbm_t* h, const Snapshot& in, const Snapshot& out, bool accumulate,
                 void* rec = nullptr) {
    Engine& e = h->e;
    e.wall_scale = e.wall_decay == 1.0 ? 1.0 : std::pow(e.wall_decay, (double)e.t);
    lbe::StepObjective so;
    const bool in_window = accumulate && e.obj_kind != LBM_OBJ_NONE &&
                           e.t >= e.obj_t0 && e.t < e.obj_t1;
    const double window = (double)(e.obj_t1 - e.obj_t0);
    if (in_window && e.obj_kind == LBM_OBJ_MEAN_UX) {
        so.acc = e.d_obj_acc;
        so.kind = LBM_OBJ_MEAN_UX;
        so.w = 1.0 / (window * (double)e.n_fluid);
    }
    if (in_window && e.obj_kind == LBM_OBJ_PRESSURE_DROP) {
        // p = c_s^2 rho with c_s^2 = 1/3
        so.acc = e.d_obj_acc;
        so.kind = LBM_OBJ_PRESSURE_DROP;
        so.w = 1.0 / (3.0 * window);
        so.x_in = (uint32_t)e.obj_x_in;
        so.x_out = (uint32_t)e.obj_x_out;
        so.a_in = e.obj_a_in;
        so.a_out = e.obj_a_out;
    }
    if (e.poison) {   // LBM_DEBUG: what the step does not write stays NaN
        HIPCHK(h, lbe::launch_fill_nan(e, out.f, (size_t)e.Q * (size_t)e.S));
        HIPCHK(h, lbe::launch_fill_nan(e, out.wa, (size_t)e.n_links));
        if (rec) HIPCHK(h, lbe::launch_fill_nan(e, rec, (size_t)lbe::record_values(e)));
    }
    HIPCHK(h, lbe::launch_step(e, in, out, so, rec));
    if (in_window && e.obj_kind == LBM_OBJ_FORCE_X)
        HIPCHK(h, lbe::launch_force_objective(e, out, e.d_obj_acc, e.obj_tag,
                                              1.0 / (double)(e.obj_t1 - e.obj_t0)));
    return LBM_OK;
}

}  // namespace

// =============================================================================
// -- reverse sweep ---------------------------------------------------------
// The sweep runs over the steps of the last checkpointed run from the last
// one backwards; adj_next is the next step to reverse (relative to run_t0),
// adj_seg the segment whose states the replay pool holds, and lam[0] holds
// lambda at the sweep's current time between calls.

namespace {

int adjoint_begin(lbm_t* h) {
    Engine& e = h->e;
    if (e.run_t0 < 0) return fail(h, LBM_ESTATE, "no checkpointed run to reverse");
    e.adj_um = e.run_urec && velocity_mode(e);
    if (e.ckpt.empty() && !e.adj_um)
        return fail(h, LBM_ESTATE,
                    "the run kept step records only (rate gradients off); "
                    "run it again with the current settings");
    if (e.two_node != e.run_two_node || (e.adj_um && e.two_node && !e.fib_final))
        return fail(h, LBM_ESTATE, "the boundary scheme changed since the run; run it again");
    int rc;
    const size_t lam_bytes = f_bytes(e);
    for (auto& l : e.lam) {
        if (!l && hipMalloc(&l, lam_bytes) != hipSuccess) {
            l = nullptr;
            return fail(h, LBM_ENOMEM, "adjoint array allocation failed");
        }
    }
    // on step records the replay of a segment records its steps but the
    // last (the run recorded that one) through two ping-pong states;
    // otherwise pool[r] holds the replayed state r of a segment (state 0 is
    // the checkpoint itself, so pool[0] stays empty)
    const int64_t seg = std::min(e.run_every, e.run_n);   // the longest segment
    if (e.adj_um && seg > 1 &&
        (rc = alloc_list(h, e.rec_pool, (size_t)(seg - 1), rec_bytes(e))))
        return rc;
    if (e.adj_um && e.two_node && !e.fib_next &&
        hipMalloc(&e.fib_next, wa_bytes(e)) != hipSuccess) {
        e.fib_next = nullptr;
        return fail(h, LBM_ENOMEM, "device allocation of link values failed");
    }
    const size_t npool = e.adj_um ? (seg > 1 ? 2 : 0) : (size_t)seg + 1;
    if (e.pool.size() != npool) {
        for (auto& s : e.pool) free_snap(s);
        e.pool.assign(npool, Snapshot{});
    }
    for (size_t k = e.adj_um ? 0 : 1; k < e.pool.size(); ++k)
        if (!e.pool[k].f && (rc = alloc_snap(h, e.pool[k]))) return rc;
    const int NC = e.D + e.Q;
    const int64_t nb = lbe::adjoint_blocks(e);
    const size_t L1 = (size_t)std::max<int64_t>(e.n_links, 1);
    if (!e.d_gq || e.gglob_len != nb || e.gq_len != (int64_t)L1) {
        free_dev(e.d_gq);
        free_dev(e.d_gglob);
        free_dev(e.ak_buf);
        free_dev(e.tq_buf);
        e.d_gs = nullptr;
        // the two per-link sums in one allocation: gq, then gs
        if (hipMalloc((void**)&e.d_gq, 2 * L1 * 8) != hipSuccess ||
            hipMalloc((void**)&e.d_gglob, (size_t)nb * NC * 8) != hipSuccess)
            return fail(h, LBM_ENOMEM, "gradient accumulator allocation failed");
        e.d_gs = e.d_gq + L1;
        e.gglob_len = nb;
        e.gq_len = (int64_t)L1;
    }
    // on records: the a_k runs of the reverse steps whose link terms pend
    if (e.adj_um && !e.ak_buf &&
        hipMalloc((void**)&e.ak_buf, (size_t)lbe::kAkBatch * L1 * 8) != hipSuccess) {
        e.ak_buf = nullptr;
        return fail(h, LBM_ENOMEM, "device allocation of the link adjoint runs failed");
    }
    if (e.adj_um && e.two_node && !e.tq_buf &&
        hipMalloc((void**)&e.tq_buf, (size_t)lbe::kAkBatch * L1 * 8) != hipSuccess) {
        e.tq_buf = nullptr;
        return fail(h, LBM_ENOMEM, "device allocation of the link adjoint runs failed");
    }
    e.ak_pending = 0;
    if ((rc = zero(h, e.d_gq, 2 * L1 * 8))) return rc;
    if ((rc = zero(h, e.d_gglob, (size_t)nb * NC * 8))) return rc;
    if ((rc = zero(h, e.lam[0], lam_bytes))) return rc;
    e.adj_next = e.run_n - 1;
    e.adj_seg = -1;
    e.adj_started = true;
    e.have_grad = true;   // partial sums are available from here on
    return LBM_OK;
}

// n more reverse steps (fewer at the start of the run)
int adjoint_steps(lbm_t* h, int64_t n) {
    Engine& e = h->e;
    const int64_t nseg = (e.run_n + e.run_every - 1) / e.run_every;
    const int64_t t_saved = e.t;
    const bool um = e.adj_um;   // fixed for the whole sweep
    int lc = 0;   // lam[lc] holds lambda(t+1)
    int rc = LBM_OK;
    for (; n > 0 && e.adj_next >= 0; --n, --e.adj_next) {
        const int64_t j = e.adj_next / e.run_every;
        const int64_t r = e.adj_next - j * e.run_every;
        const int64_t t_seg = e.run_t0 + j * e.run_every;
        const int64_t len = std::min(e.run_every, e.run_n - j * e.run_every);
        // the segment's states: the checkpoint itself, then the replayed
        // ones.  The adjoint of step r reads states r and r + 1; for
        // r = len - 1 that is the next checkpoint, so only the last segment
        // replays state len.
        auto state = [&](int64_t k) -> const Snapshot& {
            if (k == 0) return e.ckpt[j];
            if (k == len && j + 1 < nseg) return e.ckpt[j + 1];
            return e.pool[k];
        };
        if (e.adj_seg != j) {
            // Eq. (211) on records: keep f_ibar(x_f, .) at the first step of
            // segment j+1 (its record is about to be overwritten) for the
            // last step of segment j
            if (um && e.two_node && e.adj_seg == j + 1 &&
                std::min(e.run_every, e.run_n - (j + 1) * e.run_every) >= 2) {
                const hipError_t cs = hipMemcpyAsync(e.fib_next, record_links(e, e.rec_pool[0]),
                                                     wa_bytes(e), hipMemcpyDeviceToDevice,
                                                     e.stream);
                if (cs != hipSuccess) {
                    rc = fail(h, LBM_EDEVICE, std::string("link values: ") + hipGetErrorString(cs));
                    break;
                }
            }
            if (um) {
                // the pending link terms read the records about to be replaced
                const hipError_t fs = len > 1 ? lbe::launch_link_sums(e) : hipSuccess;
                if (fs != hipSuccess) {
                    rc = fail(h, LBM_EDEVICE, std::string("link sums: ") + hipGetErrorString(fs));
                    break;
                }
                // records of steps 0 .. len-2 (the run recorded step len-1)
                for (int64_t k = 0; k + 1 < len; ++k) {
                    e.t = t_seg + k;
                    const Snapshot& in = k == 0 ? e.ckpt[j] : e.pool[(k - 1) & 1];
                    if ((rc = forward_step(h, in, e.pool[k & 1], false, e.rec_pool[k]))) break;
                }
            } else {
                const int64_t nrep = j + 1 == nseg ? len : len - 1;
                for (int64_t k = 0; k < nrep; ++k) {
                    e.t = t_seg + k;   // forward_step reads e.t for the objective window and wall data
                    if ((rc = forward_step(h, state(k), e.pool[k + 1], false))) break;
                }
            }
            if (rc) break;
            e.adj_seg = j;
        }
        const int64_t t = t_seg + r;
        lbe::AdjointObjective ao;
        ao.kind = e.obj_kind;
        ao.tag = e.obj_tag;
        const bool in_w = e.obj_kind != LBM_OBJ_NONE && t >= e.obj_t0 && t < e.obj_t1;
        ao.weight = in_w ? 1.0 / (double)(e.obj_t1 - e.obj_t0) : 0.0;
        ao.inv_nfluid = e.n_fluid ? 1.0 / (double)e.n_fluid : 0.0;
        ao.x_in = (uint32_t)e.obj_x_in;
        ao.x_out = (uint32_t)e.obj_x_out;
        ao.a_in = e.obj_a_in;
        ao.a_out = e.obj_a_out;
        if (!in_w) ao.kind = LBM_OBJ_NONE;
        hipError_t st = hipSuccess;
        e.wall_scale = e.wall_decay == 1.0 ? 1.0 : std::pow(e.wall_decay, (double)t);
        if (e.poison)   // LBM_DEBUG: lambda(t) slots the step does not write stay NaN
            st = lbe::launch_fill_nan(e, e.lam[lc ^ 1], (size_t)e.Q * (size_t)e.S);
        if (e.two_node && st == hipSuccess) {
            if (um) {
                // f_ibar(x_f, t+1): the record of step t+1, or where the
                // next segment or the run ends
                const void* fibn;
                if (r + 1 < len)
                    fibn = record_links(e, r + 1 == len - 1 ? e.rec_last[j] : e.rec_pool[r + 1]);
                else if (j + 1 == nseg)
                    fibn = e.fib_final;
                else if (std::min(e.run_every, e.run_n - (j + 1) * e.run_every) >= 2)
                    fibn = e.fib_next;
                else
                    fibn = record_links(e, e.rec_last[j + 1]);
                st = lbe::launch_two_node_adjoint(e, nullptr, fibn, e.lam[lc], ao);
            } else {
                st = lbe::launch_two_node_adjoint(e, &state(r + 1), nullptr, e.lam[lc], ao);
            }
        }
        if (st == hipSuccess) {
            if (um)
                st = lbe::launch_adjoint_step(e, nullptr, nullptr,
                                              r == len - 1 ? e.rec_last[j] : e.rec_pool[r],
                                              e.lam[lc], e.lam[lc ^ 1], ao);
            else
                st = lbe::launch_adjoint_step(e, &state(r), &state(r + 1), nullptr, e.lam[lc],
                                              e.lam[lc ^ 1], ao);
        }
        if (st != hipSuccess) {
            rc = fail(h, LBM_EDEVICE, std::string("adjoint step: ") + hipGetErrorString(st));
            break;
        }
        lc ^= 1;
    }
    e.t = t_saved;
    // keep lambda at the sweep's current time in lam[0]
    if (lc != 0) std::swap(e.lam[0], e.lam[1]);
    // the sums are complete between calls
    if (rc == LBM_OK && um) {
        const hipError_t fs = lbe::launch_link_sums(e);
        if (fs != hipSuccess)
            rc = fail(h, LBM_EDEVICE, std::string("link sums: ") + hipGetErrorString(fs));
    }
    return rc;
}

}  // namespace

extern "C" {

int lbm_create(lbm_t** out, int lattice, int precision, int64_t nx, int64_t ny,
               int64_t nz, const double* s, double rho0, const double* g) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19 && lattice != LBM_D3Q15) return LBM_EINVAL;
    if (precision != LBM_FP64 && precision != LBM_FP32) return LBM_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1) return LBM_EINVAL;
    if (lattice == LBM_D2Q9 && nz != 1) return LBM_EINVAL;
    if (nx > 65535 * 256LL || ny > (1LL << 31) || nz > (1LL << 31)) return LBM_EINVAL;
    const int64_t N = nx * ny * nz;
    if (N >= (1LL << 31)) return LBM_EINVAL;
    // one direction plane must stay below 4 GiB (32-bit byte offsets)
    if (N * (precision == LBM_FP64 ? 8 : 4) >= (1LL << 32)) return LBM_EINVAL;
    if (!s || !(rho0 > 0.0) || !std::isfinite(rho0)) return LBM_EINVAL;
    const int Q = lat_Q(lattice), D = lat_D(lattice);
    for (int k = 0; k < Q; ++k) {
        if (!std::isfinite(s[k])) return LBM_EINVAL;
        if (!lat_conserved(lattice, k) && !(s[k] >= 0.0 && s[k] < 2.0)) return LBM_EINVAL;
    }
    if (g)
        for (int a = 0; a < D; ++a)
            if (!std::isfinite(g[a])) return LBM_EINVAL;

    lbm_t* h = new (std::nothrow) lbm_t;
    if (!h) return LBM_ENOMEM;
    Engine& e = h->e;
    e.lattice = lattice;
    e.precision = precision;
    e.Q = Q;
    e.D = D;
    e.nx = nx;
    e.ny = ny;
    e.nz = nz;
    e.N = N;
    e.elem = precision == LBM_FP64 ? 8 : 4;
    e.S = plane_stride(N);
    if (e.S * (int64_t)e.elem >= (1LL << 32)) {
        delete h;
        return LBM_EINVAL;
    }
    // launch-bound sizes replay graphs of 64 steps (LBM_GRAPH_STEPS overrides;
    // an even count, 0 disables)
    e.graph_steps = N <= (1LL << 20) ? 64 : 0;
    if (const char* v = std::getenv("LBM_GRAPH_STEPS")) {
        const int gsteps = std::atoi(v);
        e.graph_steps = gsteps > 0 ? (gsteps + 1) / 2 * 2 : 0;
    }
    // LBM_DEBUG=1: poison mode (every step's outputs are filled with NaN
    // first, so a read of a slot the previous step did not write shows up
    // as a non-finite reduction); steps are launched one by one
    if (const char* v = std::getenv("LBM_DEBUG")) e.poison = std::atoi(v) != 0;
    if (e.poison) e.graph_steps = 0;
    for (int k = 0; k < Q; ++k) e.s[k] = s[k];
    e.rho0 = rho0;
    for (int a = 0; a < 3; ++a) e.g[a] = (g && a < D) ? g[a] : 0.0;
    if (hipGetDevice(&e.device) != hipSuccess) {
        delete h;
        return LBM_EDEVICE;
    }
    if (hipStreamCreate(&e.own_stream) != hipSuccess) {
        delete h;
        return LBM_EDEVICE;
    }
    e.stream = e.own_stream;
    for (auto& b : e.buf) {
        if (hipMalloc(&b.f, f_bytes(e)) != hipSuccess) {
            b.f = nullptr;
            lbm_destroy(h);
            return LBM_ENOMEM;
        }
        if (hipMemsetAsync(b.f, 0, f_bytes(e), e.stream) != hipSuccess) {
            lbm_destroy(h);
            return LBM_EDEVICE;
        }
    }
    if (hipEventCreate(&e.ev0) != hipSuccess || hipEventCreate(&e.ev1) != hipSuccess) {
        lbm_destroy(h);
        return LBM_EDEVICE;
    }
    *out = h;
    return LBM_OK;
}

int lbm_set_scheme(lbm_t* h, int l_rule, double b) {
    if (!h) return LBM_EINVAL;
    if (l_rule < LBM_L_GAMMA || l_rule > LBM_L_MIN)
        return fail(h, LBM_EINVAL, "unknown l rule");
    if (!(b > 0.0 && b <= 1.0)) return fail(h, LBM_EINVAL, "b must lie in (0, 1]");
    if (h->e.has_geometry) return fail(h, LBM_ESTATE, "set the scheme before the geometry");
    h->e.l_rule = l_rule;
    h->e.b = b;
    return LBM_OK;
}

int lbm_set_two_node(lbm_t* h, int on) {
    if (!h) return LBM_EINVAL;
    if (h->e.has_geometry) return fail(h, LBM_ESTATE, "choose the variant before the geometry");
    h->e.two_node = on != 0;
    return LBM_OK;
}

int lbm_set_wall_decay(lbm_t* h, double lambda) {
    if (!h) return LBM_EINVAL;
    if (!std::isfinite(lambda) || !(lambda > 0.0))
        return fail(h, LBM_EINVAL, "wall decay factor must be finite and positive");
    h->e.wall_decay = lambda;
    return LBM_OK;
}

int lbm_set_x_boundary(lbm_t* h, int kind, double drho) {
    if (!h) return LBM_EINVAL;
    if (kind < LBM_X_PERIODIC || kind > LBM_X_OUTFLOW)
        return fail(h, LBM_EINVAL, "unknown x boundary kind");
    if (!std::isfinite(drho)) return fail(h, LBM_EINVAL, "drho must be finite");
    if (h->e.has_geometry)
        return fail(h, LBM_ESTATE, "set the x boundary before the geometry");
    h->e.xbc = kind;
    h->e.drho = drho;
    return LBM_OK;
}

int lbm_set_geometry(lbm_t* h, const uint8_t* solid, int64_t n_links,
                     const int64_t* node, const int8_t* dir, const double* q,
                     const double* wall_u, const int32_t* tag) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    // validation, link sort and the node / wave tables (host, geometry.cpp)
    int E[19][3];
    for (int i = 0; i < e.Q; ++i)
        for (int a = 0; a < 3; ++a) E[i][a] = a < e.D ? lat_e(e.lattice, i, a) : 0;
    lbe::GeomDomain dom;
    dom.Q = e.Q;
    dom.D = e.D;
    dom.e = E;
    dom.nx = e.nx;
    dom.ny = e.ny;
    dom.nz = e.nz;
    dom.outflow = e.xbc == LBM_X_OUTFLOW;
    dom.block = lbe::kBlock;
    dom.wave = lbe::kWave;
    lbe::GeomLinks links;
    links.n = n_links;
    links.node = node;
    links.dir = dir;
    links.q = q;
    links.wall_u = wall_u;
    links.tag = tag;
    lbe::GeomTables tab;
    std::string why;
    const int vrc = lbe::build_geometry(dom, solid, links, tab, why);
    if (vrc) return fail(h, vrc, why);
    static_assert(sizeof(lbe::WaveWord) == sizeof(uint2) && sizeof(lbe::WaveEntry) == sizeof(uint4),
                  "host wave tables must match the device vector types");
    e.perm = tab.perm;
    e.n_links = n_links;
    e.n_fluid = tab.n_fluid;
    e.fluid_per_x = tab.fluid_per_x;
    e.obj_kind = LBM_OBJ_NONE;   // an objective refers to the previous geometry
    e.lk_node_h = tab.node;
    e.lk_dir_h = tab.dir;
    e.q_h = tab.q;
    e.wall_u_h = tab.wall_u;
    e.tag_h = tab.tag;
    e.n_tags = tab.n_tags;
    e.ibar_is_link = tab.ibar_is_link;
    const std::vector<uint32_t>& info = tab.info;
    const auto* wave = reinterpret_cast<const uint2*>(tab.wave.data());
    const auto* wact = reinterpret_cast<const uint4*>(tab.wact.data());
    e.n_wact = (int64_t)tab.wact.size();
    std::vector<uint8_t> d8(n_links);
    std::vector<int32_t> n32(n_links);
    for (int64_t k = 0; k < n_links; ++k) {
        d8[k] = (uint8_t)e.lk_dir_h[k];
        n32[k] = (int32_t)e.lk_node_h[k];
    }
    e.has_geometry = false;
    drop_graphs(e);
    free_run(e);
    int rc;
    if ((rc = upload(h, e.d_info, info.data(), info.size()))) return rc;
    if ((rc = upload(h, e.d_wave, wave, tab.wave.size()))) return rc;
    if ((rc = upload(h, e.d_wact, wact, tab.wact.size()))) return rc;
    if ((rc = upload(h, e.d_lkdir, d8.data(), d8.size()))) return rc;
    if ((rc = upload(h, e.d_lknode, n32.data(), n32.size()))) return rc;
    {
        std::vector<int32_t> p32(n_links);
        for (int64_t k = 0; k < n_links; ++k) p32[k] = (int32_t)e.perm[k];
        if ((rc = upload(h, e.d_perm, p32.data(), p32.size()))) return rc;
    }
    if ((rc = upload(h, e.d_lktag, e.tag_h.data(), e.tag_h.size()))) return rc;
    if ((rc = upload_coefficients(h))) return rc;
    for (auto& b : e.buf) {
        if (b.wa) (void)hipFree(b.wa);
        if (hipMalloc(&b.wa, wa_bytes(e)) != hipSuccess) {
            b.wa = nullptr;
            return fail(h, LBM_ENOMEM, "device allocation of link slots failed");
        }
        if ((rc = zero(h, b.wa, wa_bytes(e)))) return rc;
    }
    e.has_geometry = true;
    e.initialized = false;
    e.have_grad = false;
    e.adj_started = false;
    return sync(h);
}

int lbm_update_links(lbm_t* h, const double* q, const double* wall_u) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.has_geometry) return fail(h, LBM_ESTATE, "no geometry");
    std::vector<double> q_old = e.q_h, u_old = e.wall_u_h;
    for (int64_t k = 0; k < e.n_links; ++k) {
        const int64_t p = e.perm[k];
        if (q) {
            if (!(q[p] > 0.0 && q[p] <= 1.0)) {
                e.q_h = q_old;
                return fail(h, LBM_EINVAL, "q must lie in (0, 1]");
            }
            e.q_h[k] = q[p];
        }
        if (wall_u)
            for (int a = 0; a < e.D; ++a) e.wall_u_h[k * e.D + a] = wall_u[p * e.D + a];
    }
    HIPCHK(h, hipStreamSynchronize(e.stream));
    drop_graphs(e);
    const int rc = upload_coefficients(h);
    if (rc) {
        e.q_h = q_old;
        e.wall_u_h = u_old;
    }
    return rc;
}

int lbm_set_parameters(lbm_t* h, const double* s, const double* g) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (s)
        for (int k = 0; k < e.Q; ++k) {
            if (!std::isfinite(s[k])) return fail(h, LBM_EINVAL, "rate not finite");
            if (!lat_conserved(e.lattice, k) && !(s[k] >= 0.0 && s[k] < 2.0))
                return fail(h, LBM_EINVAL, "relaxation rates must lie in [0, 2)");
        }
    if (g)
        for (int a = 0; a < e.D; ++a)
            if (!std::isfinite(g[a])) return fail(h, LBM_EINVAL, "force not finite");
    HIPCHK(h, hipStreamSynchronize(e.stream));
    drop_graphs(e);
    if (s)
        for (int k = 0; k < e.Q; ++k) e.s[k] = s[k];
    if (g)
        for (int a = 0; a < e.D; ++a) e.g[a] = g[a];
    return LBM_OK;
}

int lbm_collision_rates(int lattice, int kind, double s_nu, double magic, double* s_out) {
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19 && lattice != LBM_D3Q15) return LBM_EINVAL;
    if (!s_out || !(s_nu > 0.0 && s_nu < 2.0)) return LBM_EINVAL;
    if (kind != LBM_COLLISION_BGK && kind != LBM_COLLISION_TRT) return LBM_EINVAL;
    double s_minus = s_nu;
    if (kind == LBM_COLLISION_TRT) {
        if (!(magic > 0.0) || !std::isfinite(magic)) return LBM_EINVAL;
        s_minus = 1.0 / (0.5 + magic / (1.0 / s_nu - 0.5));
    }
    const int Q = lat_Q(lattice), D = lat_D(lattice);
    for (int k = 0; k < Q; ++k) {
        // row k is even when M[k][ibar] = M[k][i] for every direction i
        bool even = true;
        for (int i = 0; i < Q; ++i) {
            int ib = 0;
            for (int j = 0; j < Q; ++j) {
                bool opp = true;
                for (int a = 0; a < D; ++a) opp = opp && lat_e(lattice, j, a) == -lat_e(lattice, i, a);
                if (opp) ib = j;
            }
            even = even && lat_M(lattice, k, ib) == lat_M(lattice, k, i);
        }
        s_out[k] = even ? s_nu : s_minus;
    }
    return LBM_OK;
}

int lbm_set_collision(lbm_t* h, int kind, double s_nu, double magic) {
    if (!h) return LBM_EINVAL;
    double s[19];
    const int rc = lbm_collision_rates(h->e.lattice, kind, s_nu, magic, s);
    if (rc) return fail(h, rc, "collision: kind must be BGK or TRT, s_nu in (0, 2), magic > 0");
    return lbm_set_parameters(h, s, nullptr);
}

static int init_common(lbm_t* h, const double* df, const double* rho, const double* u) {
    Engine& e = h->e;
    if (!e.has_geometry) return fail(h, LBM_ESTATE, "set the geometry before init");
    int64_t need = 0;
    if (df) need = (int64_t)e.Q * e.N;
    else need = (rho ? e.N : 0) + (u ? e.N * e.D : 0);
    int rc = ensure_scratch(h, std::max<int64_t>(need, 1));
    if (rc) return rc;
    double* d_df = nullptr;
    double* d_rho = nullptr;
    double* d_u = nullptr;
    if (df) {
        d_df = e.d_scratch;
        HIPCHK(h, hipMemcpyAsync(d_df, df, (size_t)need * 8, hipMemcpyHostToDevice, e.stream));
    } else {
        double* p = e.d_scratch;
        if (rho) {
            d_rho = p;
            HIPCHK(h, hipMemcpyAsync(d_rho, rho, (size_t)e.N * 8, hipMemcpyHostToDevice, e.stream));
            p += e.N;
        }
        if (u) {
            d_u = p;
            HIPCHK(h, hipMemcpyAsync(d_u, u, (size_t)e.N * e.D * 8, hipMemcpyHostToDevice, e.stream));
        }
    }
    Snapshot& s = e.buf[e.cur];
    if ((rc = zero(h, s.f, f_bytes(e)))) return rc;
    if ((rc = zero(h, s.wa, wa_bytes(e)))) return rc;
    HIPCHK(h, lbe::launch_init(e, d_df, d_rho, d_u, s));
    e.t = 0;
    e.initialized = true;
    e.stepped = false;
    return sync(h);
}

int lbm_init(lbm_t* h, const double* rho, const double* u) {
    if (!h) return LBM_EINVAL;
    return init_common(h, nullptr, rho, u);
}

int lbm_init_deviation(lbm_t* h, const double* df) {
    if (!h || !df) return LBM_EINVAL;
    return init_common(h, df, nullptr, nullptr);
}

int lbm_step(lbm_t* h, int64_t n) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (n < 0) return fail(h, LBM_EINVAL, "negative step count");
    if (!e.initialized) return fail(h, LBM_ESTATE, "initialise before stepping");
    if (e.timing && n > 0) HIPCHK(h, hipEventRecord(e.ev0, e.stream));
    int64_t left = n;
    // small domains are launch-bound: replay captured loops of graph_steps
    // steps while no objective window is open
    const bool obj_open = e.obj_kind != LBM_OBJ_NONE && e.t < e.obj_t1 && e.t + n > e.obj_t0;
    if (e.graph_steps > 0 && !obj_open && e.wall_decay == 1.0) {
        while (left >= e.graph_steps) {
            if (!e.graph_exec[e.cur]) {
                const int rc = build_graph(h, e.cur);
                if (rc) return rc;
            }
            HIPCHK(h, hipGraphLaunch(e.graph_exec[e.cur], e.stream));
            e.t += e.graph_steps;
            left -= e.graph_steps;
            e.stepped = true;
        }
    }
    for (; left > 0; --left) {
        const int rc = forward_step(h, e.buf[e.cur], e.buf[e.cur ^ 1], true);
        if (rc) return rc;
        e.cur ^= 1;
        ++e.t;
        e.stepped = true;
    }
    if (e.timing && n > 0) {
        HIPCHK(h, hipEventRecord(e.ev1, e.stream));
        e.timed_steps = n;        // resolved in lbm_last_step_ms
    }
    return LBM_OK;
}

int64_t lbm_time(const lbm_t* h) { return h ? h->e.t : -1; }

int lbm_moments(lbm_t* h, double* rho, double* u) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.initialized) return fail(h, LBM_ESTATE, "not initialised");
    const int64_t need = e.N * (1 + e.D);
    int rc = ensure_scratch(h, need);
    if (rc) return rc;
    double* d_rho = e.d_scratch;
    double* d_u = e.d_scratch + e.N;
    HIPCHK(h, lbe::launch_observe(e, e.buf[e.cur], d_rho, d_u, nullptr));
    if (rho) HIPCHK(h, hipMemcpyAsync(rho, d_rho, (size_t)e.N * 8, hipMemcpyDeviceToHost, e.stream));
    if (u) HIPCHK(h, hipMemcpyAsync(u, d_u, (size_t)e.N * e.D * 8, hipMemcpyDeviceToHost, e.stream));
    return sync(h);
}

int lbm_get_distribution(lbm_t* h, double* df) {
    if (!h || !df) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.initialized) return fail(h, LBM_ESTATE, "not initialised");
    const int64_t need = (int64_t)e.Q * e.N;
    int rc = ensure_scratch(h, need);
    if (rc) return rc;
    HIPCHK(h, lbe::launch_observe(e, e.buf[e.cur], nullptr, nullptr, e.d_scratch));
    HIPCHK(h, hipMemcpyAsync(df, e.d_scratch, (size_t)need * 8, hipMemcpyDeviceToHost, e.stream));
    return sync(h);
}

int lbm_reduce(lbm_t* h, double* mass, double* mom) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.initialized) return fail(h, LBM_ESTATE, "not initialised");
    const int64_t nb = lbe::step_blocks(e);
    const int cols = 1 + e.D;
    int rc = ensure_scratch(h, nb * cols + cols);
    if (rc) return rc;
    int64_t rows = 0;
    HIPCHK(h, lbe::launch_mass(e, e.buf[e.cur], e.d_scratch, &rows));
    double* d_out = e.d_scratch + nb * cols;
    HIPCHK(h, lbe::launch_sum_blocks(e, e.d_scratch, rows, cols, d_out));
    double out[4] = {0, 0, 0, 0};
    HIPCHK(h, hipMemcpyAsync(out, d_out, cols * 8, hipMemcpyDeviceToHost, e.stream));
    if ((rc = sync(h))) return rc;
    const double m = (double)e.n_fluid * e.rho0 + out[0];
    if (mass) *mass = m;
    if (mom)
        for (int a = 0; a < e.D; ++a) mom[a] = out[1 + a];
    bool finite = std::isfinite(m);
    for (int a = 0; a < e.D; ++a) finite = finite && std::isfinite(out[1 + a]);
    if (!finite) return fail(h, LBM_ENONFINITE, "mass or momentum is not finite");
    return LBM_OK;
}

int lbm_reduce_noalloc(lbm_t* h, double* mass, double* mom) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.initialized) return fail(h, LBM_ESTATE, "not initialised");
    const int64_t nb = lbe::step_blocks(e);
    const int cols = 1 + e.D;
    if (nb * cols + cols > lbe::kNoAllocScratchDoubles)
        return fail(h, LBM_EINVAL,
                    "domain too large for the fixed reduction scratch: " +
                        std::to_string(nb * cols + cols) + " partial sums needed, at most " +
                        std::to_string(lbe::kNoAllocScratchDoubles) + " (" +
                        std::to_string((lbe::kNoAllocScratchDoubles / cols - 1) * lbe::kBlock) +
                        " nodes)");
    double* scr = nullptr;
    HIPCHK(h, lbe::noalloc_scratch(e.device, &scr));
    int64_t rows = 0;
    HIPCHK(h, lbe::launch_mass(e, e.buf[e.cur], scr, &rows));
    double* d_out = scr + nb * cols;
    HIPCHK(h, lbe::launch_sum_blocks(e, scr, rows, cols, d_out));
    double out[4] = {0, 0, 0, 0};
    HIPCHK(h, hipMemcpyAsync(out, d_out, cols * 8, hipMemcpyDeviceToHost, e.stream));
    int rc = sync(h);
    if (rc) return rc;
    const double m = (double)e.n_fluid * e.rho0 + out[0];
    if (mass) *mass = m;
    if (mom)
        for (int a = 0; a < e.D; ++a) mom[a] = out[1 + a];
    bool finite = std::isfinite(m);
    for (int a = 0; a < e.D; ++a) finite = finite && std::isfinite(out[1 + a]);
    if (!finite) return fail(h, LBM_ENONFINITE, "mass or momentum is not finite");
    return LBM_OK;
}

int lbm_force(lbm_t* h, int32_t n_tags, double* force) {
    if (!h || !force || n_tags < 0) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.stepped) return fail(h, LBM_ESTATE, "no step taken yet");
    const int D = e.D;
    for (int64_t c = 0; c < (int64_t)n_tags * D; ++c) force[c] = 0.0;
    if (e.n_links == 0 || e.n_tags == 0) return LBM_OK;
    const int64_t nb = lbe::link_blocks(e);
    const int64_t cols = (int64_t)e.n_tags * D;
    int rc = ensure_scratch(h, nb * cols + cols);
    if (rc) return rc;
    int64_t rows = 0;
    HIPCHK(h, lbe::launch_force(e, e.buf[e.cur], e.d_scratch, &rows));
    double* d_out = e.d_scratch + nb * cols;
    HIPCHK(h, lbe::launch_sum_blocks(e, e.d_scratch, rows, cols, d_out));
    std::vector<double> out(cols);
    HIPCHK(h, hipMemcpyAsync(out.data(), d_out, cols * 8, hipMemcpyDeviceToHost, e.stream));
    if ((rc = sync(h))) return rc;
    for (int t = 0; t < std::min<int>(n_tags, e.n_tags); ++t)
        for (int a = 0; a < D; ++a) force[t * D + a] = out[t * D + a];
    return LBM_OK;
}

int64_t lbm_state_bytes(const lbm_t* h) {
    if (!h || !h->e.has_geometry) return -1;
    return (int64_t)(f_bytes(h->e) + wa_bytes(h->e));
}

int lbm_get_state(lbm_t* h, void* dst) {
    if (!h || !dst) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.initialized) return fail(h, LBM_ESTATE, "not initialised");
    Snapshot d{dst, (char*)dst + f_bytes(e)};
    int rc = copy_snap(h, d, e.buf[e.cur]);
    if (rc) return rc;
    return sync(h);
}

int lbm_set_state(lbm_t* h, const void* src, int64_t time) {
    if (!h || !src || time < 0) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.has_geometry) return fail(h, LBM_ESTATE, "set the geometry first");
    Snapshot s{(void*)src, (char*)src + f_bytes(e)};
    int rc = copy_snap(h, e.buf[e.cur], s);
    if (rc) return rc;
    e.t = time;
    e.initialized = true;
    e.stepped = time > 0;
    return sync(h);
}

int lbm_set_objective(lbm_t* h, int kind, int32_t tag, int64_t t_begin, int64_t t_end) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (kind < LBM_OBJ_NONE || kind > LBM_OBJ_PRESSURE_DROP)
        return fail(h, LBM_EINVAL, "unknown objective");
    if (kind != LBM_OBJ_NONE && !(t_end > t_begin && t_begin >= 0))
        return fail(h, LBM_EINVAL, "objective window must satisfy 0 <= t_begin < t_end");
    if (!e.has_geometry) return fail(h, LBM_ESTATE, "set the geometry first");
    if (kind == LBM_OBJ_FORCE_X && (tag < 0 || tag >= e.n_tags))
        return fail(h, LBM_EINVAL, "objective tag has no links");
    if (kind == LBM_OBJ_PRESSURE_DROP) {
        const int64_t xo = e.obj_x_out < 0 ? e.nx - 1 : e.obj_x_out;
        const int64_t ni = e.fluid_per_x[e.obj_x_in], no = e.fluid_per_x[xo];
        if (ni == 0 || no == 0)
            return fail(h, LBM_EINVAL, "a pressure-drop plane has no fluid node");
        e.obj_x_out = xo;
        e.obj_a_in = 1.0 / (double)ni;
        e.obj_a_out = 1.0 / (double)no;
    }
    e.obj_kind = kind;
    e.obj_tag = tag;
    e.obj_t0 = t_begin;
    e.obj_t1 = t_end;
    const int64_t len = kind == LBM_OBJ_FORCE_X ? lbe::link_blocks(e) : lbe::step_blocks(e);
    free_dev(e.d_obj_acc);
    e.obj_acc_len = 0;
    if (kind != LBM_OBJ_NONE) {
        if (hipMalloc((void**)&e.d_obj_acc, (size_t)std::max<int64_t>(len, 1) * 8) != hipSuccess) {
            e.d_obj_acc = nullptr;
            return fail(h, LBM_ENOMEM, "objective accumulator allocation failed");
        }
        e.obj_acc_len = len;
        int rc = zero(h, e.d_obj_acc, (size_t)std::max<int64_t>(len, 1) * 8);
        if (rc) return rc;
    }
    return sync(h);
}

int lbm_set_objective_planes(lbm_t* h, int64_t x_in, int64_t x_out) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (x_in < 0 || x_in >= e.nx || x_out < 0 || x_out >= e.nx)
        return fail(h, LBM_EINVAL, "pressure-drop planes must lie in [0, nx)");
    e.obj_x_in = x_in;
    e.obj_x_out = x_out;
    return LBM_OK;
}

int lbm_pressure_drop(lbm_t* h, int64_t x_in, int64_t x_out, double* dp) {
    if (!h || !dp) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.initialized) return fail(h, LBM_ESTATE, "not initialised");
    if (x_in < 0 || x_in >= e.nx || x_out < 0 || x_out >= e.nx)
        return fail(h, LBM_EINVAL, "pressure-drop planes must lie in [0, nx)");
    const int64_t ni = e.fluid_per_x[x_in], no = e.fluid_per_x[x_out];
    if (ni == 0 || no == 0) return fail(h, LBM_EINVAL, "a pressure-drop plane has no fluid node");
    const int64_t nb = (2 * e.ny * e.nz + lbe::kBlock - 1) / lbe::kBlock;
    int rc = ensure_scratch(h, nb + 1);
    if (rc) return rc;
    int64_t rows = 0;
    HIPCHK(h, lbe::launch_plane_density(e, e.buf[e.cur], (uint32_t)x_in, (uint32_t)x_out,
                                        1.0 / (double)ni, 1.0 / (double)no, e.d_scratch, &rows));
    HIPCHK(h, lbe::launch_sum_blocks(e, e.d_scratch, rows, 1, e.d_scratch + nb));
    double out = 0.0;
    HIPCHK(h, hipMemcpyAsync(&out, e.d_scratch + nb, 8, hipMemcpyDeviceToHost, e.stream));
    if ((rc = sync(h))) return rc;
    *dp = out / 3.0;   // p = c_s^2 rho
    if (!std::isfinite(*dp)) return fail(h, LBM_ENONFINITE, "pressure drop is not finite");
    return LBM_OK;
}

int lbm_objective(lbm_t* h, double* J) {
    if (!h || !J) return LBM_EINVAL;
    Engine& e = h->e;
    *J = 0.0;
    if (e.obj_kind == LBM_OBJ_NONE || e.obj_acc_len == 0) return LBM_OK;
    int rc = ensure_scratch(h, 1);
    if (rc) return rc;
    HIPCHK(h, lbe::launch_sum_blocks(e, e.d_obj_acc, e.obj_acc_len, 1, e.d_scratch));
    HIPCHK(h, hipMemcpyAsync(J, e.d_scratch, 8, hipMemcpyDeviceToHost, e.stream));
    if ((rc = sync(h))) return rc;
    if (!std::isfinite(*J)) return fail(h, LBM_ENONFINITE, "objective is not finite");
    return LBM_OK;
}

int lbm_run_checkpointed(lbm_t* h, int64_t n, int64_t every) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.initialized) return fail(h, LBM_ESTATE, "initialise before running");
    if (n < 1 || every < 1) return fail(h, LBM_EINVAL, "n and every must be >= 1");
    // checkpoint buffers are kept between runs of the same length (the
    // replay pool and adjoint arrays are kept by lbm_adjoint likewise).  A
    // sweep on step records needs no snapshot for segments of one step.
    const int64_t nseg = (n + every - 1) / every;
    const bool urec = velocity_mode(e);
    const int64_t nck = urec && every == 1 ? 0 : nseg;
    if ((int64_t)e.ckpt.size() != nck) {
        free_run(e);
        e.ckpt.resize(nck);
        for (auto& s : e.ckpt) {
            int rc = alloc_snap(h, s);
            if (rc) {
                free_run(e);
                return rc;
            }
        }
    }
    e.run_t0 = e.t;
    e.run_n = n;
    e.run_every = every;
    // the record of each segment's last step, for a reverse sweep on step
    // records (the replay records the others)
    e.run_urec = urec;
    e.run_two_node = e.two_node;
    if (urec) {
        const int rc = alloc_list(h, e.rec_last, (size_t)nseg, rec_bytes(e));
        if (rc) {
            e.run_urec = false;
            e.run_t0 = -1;
            return rc;
        }
    } else {
        free_list(e.rec_last);
    }
    // a checkpoint takes the current state's buffers (the state it must
    // keep) and hands its own, unused ones to the ping-pong pair: no copies
    drop_graphs(e);
    for (int64_t s = 0; s < n; ++s) {
        int rc;
        const Snapshot* in = &e.buf[e.cur];
        if (nck && s % every == 0) {
            std::swap(e.ckpt[s / every], e.buf[e.cur]);
            in = &e.ckpt[s / every];
        }
        const bool seg_end = (s + 1) % every == 0 || s + 1 == n;
        void* rec = urec && seg_end ? e.rec_last[s / every] : nullptr;
        if ((rc = forward_step(h, *in, e.buf[e.cur ^ 1], true, rec))) {
            e.run_t0 = -1;   // no sweep over a run that did not finish
            return rc;
        }
        e.cur ^= 1;
        ++e.t;
        e.stepped = true;
    }
    // Eq. (211) on records: f_ibar(x_f, t) of every link at the final state,
    // for the run's last reverse step
    if (urec && e.two_node) {
        if (!e.fib_final && hipMalloc(&e.fib_final, wa_bytes(e)) != hipSuccess) {
            e.fib_final = nullptr;
            e.run_t0 = -1;
            return fail(h, LBM_ENOMEM, "device allocation of link values failed");
        }
        const hipError_t st = lbe::launch_link_pull(e, e.buf[e.cur], e.fib_final);
        if (st != hipSuccess) {
            e.run_t0 = -1;
            return fail(h, LBM_EDEVICE, std::string("link values: ") + hipGetErrorString(st));
        }
    }
    e.have_grad = false;
    e.adj_started = false;
    return LBM_OK;
}


int lbm_adjoint(lbm_t* h) {
    if (!h) return LBM_EINVAL;
    const int rc = adjoint_begin(h);
    if (rc) return rc;
    return adjoint_steps(h, h->e.run_n);
}

int lbm_adjoint_step(lbm_t* h, int64_t n) {
    if (!h) return LBM_EINVAL;
    if (n < 0) return fail(h, LBM_EINVAL, "n must be >= 0");
    if (!h->e.adj_started) {
        const int rc = adjoint_begin(h);
        if (rc) return rc;
    }
    return adjoint_steps(h, n);
}

int64_t lbm_adjoint_remaining(const lbm_t* h) {
    if (!h || !h->e.adj_started) return -1;
    return h->e.adj_next + 1;
}

int lbm_set_rate_gradient(lbm_t* h, int on) {
    if (!h) return LBM_EINVAL;
    h->e.want_ds = on != 0;
    return LBM_OK;
}

int lbm_grad(lbm_t* h, double* dq, double* dwall_u, double* dg, double* ds) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.have_grad) return fail(h, LBM_ESTATE, "run lbm_adjoint first");
    const int D = e.D, Q = e.Q, NC = D + Q;
    const int64_t L = e.n_links;
    int rc;
    // scratch: [global sums NC][dq L][dphi L*D], the per-link ones already in
    // the caller's order
    if ((rc = ensure_scratch(h, NC + L * (1 + D)))) return rc;
    double* d_dq = e.d_scratch + NC;
    double* d_dphi = d_dq + L;
    HIPCHK(h, lbe::launch_sum_blocks(e, e.d_gglob, e.gglob_len, NC, e.d_scratch));
    HIPCHK(h, lbe::launch_link_gradients(e, dq ? d_dq : nullptr, dwall_u ? d_dphi : nullptr));
    std::vector<double> glob(NC);
    HIPCHK(h, hipMemcpyAsync(glob.data(), e.d_scratch, NC * 8, hipMemcpyDeviceToHost, e.stream));
    if (dq && L) HIPCHK(h, hipMemcpyAsync(dq, d_dq, L * 8, hipMemcpyDeviceToHost, e.stream));
    if (dwall_u && L)
        HIPCHK(h, hipMemcpyAsync(dwall_u, d_dphi, L * D * 8, hipMemcpyDeviceToHost, e.stream));
    if ((rc = sync(h))) return rc;
    if (dg)
        for (int a = 0; a < D; ++a) dg[a] = glob[a];
    if (ds)
        for (int k = 0; k < Q; ++k) ds[k] = glob[D + k];
    return LBM_OK;
}

int lbm_grad_device(lbm_t* h, void* dq_dev, void* dwall_u_dev, double* dg, double* ds) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.have_grad) return fail(h, LBM_ESTATE, "run lbm_adjoint first");
    HIPCHK(h, lbe::launch_link_gradients(e, (double*)dq_dev, (double*)dwall_u_dev));
    if (!dg && !ds) return LBM_OK;
    return lbm_grad(h, nullptr, nullptr, dg, ds);
}

int lbm_get_adjoint(lbm_t* h, double* lam) {
    if (!h || !lam) return LBM_EINVAL;
    Engine& e = h->e;
    if (!e.have_grad) return fail(h, LBM_ESTATE, "run lbm_adjoint first");
    const int64_t need = (int64_t)e.Q * e.N;
    int rc = ensure_scratch(h, need);
    if (rc) return rc;
    HIPCHK(h, lbe::launch_adjoint_out(e, e.lam[0], e.d_scratch));
    HIPCHK(h, hipMemcpyAsync(lam, e.d_scratch, (size_t)need * 8, hipMemcpyDeviceToHost, e.stream));
    return sync(h);
}

int lbm_set_stream(lbm_t* h, void* stream) {
    if (!h) return LBM_EINVAL;
    Engine& e = h->e;
    HIPCHK(h, hipStreamSynchronize(e.stream));
    drop_graphs(e);
    e.stream = stream ? (hipStream_t)stream : e.own_stream;
    return LBM_OK;
}

int lbm_lattice_info(int lattice, int32_t* Q, int32_t* D, int8_t* e, double* w,
                     double* M) {
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19 && lattice != LBM_D3Q15) return LBM_EINVAL;
    const int q = lat_Q(lattice), d = lat_D(lattice);
    if (Q) *Q = q;
    if (D) *D = d;
    for (int i = 0; i < q; ++i) {
        if (e)
            for (int a = 0; a < d; ++a) e[i * d + a] = (int8_t)lat_e(lattice, i, a);
        if (w) w[i] = lat_w(lattice, i);
    }
    if (M)
        for (int k = 0; k < q; ++k)
            for (int i = 0; i < q; ++i) M[k * q + i] = lat_M(lattice, k, i);
    return LBM_OK;
}

int lbm_counts(const lbm_t* h, int64_t* n_fluid, int64_t* n_links) {
    if (!h) return LBM_EINVAL;
    if (n_fluid) *n_fluid = h->e.n_fluid;
    if (n_links) *n_links = h->e.n_links;
    return LBM_OK;
}

int lbm_set_timing(lbm_t* h, int on) {
    if (!h) return LBM_EINVAL;
    h->e.timing = on != 0;
    return LBM_OK;
}

int lbm_last_step_ms(lbm_t* h, double* ms) {
    if (!h || !ms) return LBM_EINVAL;
    Engine& e = h->e;
    if (e.timed_steps > 0) {
        HIPCHK(h, hipEventSynchronize(e.ev1));
        float el = 0.f;
        HIPCHK(h, hipEventElapsedTime(&el, e.ev0, e.ev1));
        e.last_ms = (double)el / (double)e.timed_steps;
        e.timed_steps = 0;
    }
    if (e.last_ms < 0) return fail(h, LBM_ESTATE, "no timed lbm_step call");
    *ms = e.last_ms;
    return LBM_OK;
}

const char* lbm_last_error(const lbm_t* h) { return h ? h->e.err.c_str() : "null handle"; }

int lbm_destroy(lbm_t* h) {
    if (!h) return LBM_OK;
    Engine& e = h->e;
    if (e.stream) (void)hipStreamSynchronize(e.stream);
    drop_graphs(e);
    free_run(e);
    for (auto& b : e.buf) free_snap(b);
    free_dev(e.d_info);
    free_dev(e.d_wave);
    free_dev(e.d_wact);
    free_dev(e.d_lkdir);
    free_dev(e.d_lknode);
    free_dev(e.d_perm);
    free_dev(e.d_lktag);
    free_dev(e.d_lkcoef);
    free_dev(e.d_lkcoef_f);
    free_dev(e.d_lkderiv);
    free_dev(e.d_lkc4);
    free_dev(e.d_lkc1d);
    free_dev(e.d_lkd1d);
    free_dev(e.d_obj_acc);
    free_dev(e.d_gq);
    e.d_gs = nullptr;
    free_dev(e.d_gglob);
    free_dev(e.ak_buf);
    free_dev(e.tq_buf);
    free_dev(e.d_scratch);
    if (e.ev0) (void)hipEventDestroy(e.ev0);
    if (e.ev1) (void)hipEventDestroy(e.ev1);
    if (e.own_stream) (void)hipStreamDestroy(e.own_stream);
    delete h;
    return LBM_OK;
}

}  // extern "C"
