// Host-side state of one solver handle and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace lbe {

constexpr int kBlock = 256;             // threads per block of node launches
constexpr int kWave = 64;
// doubles of the fixed per-device scratch of the allocation-free entry points
// (4 MiB)
constexpr int64_t kNoAllocScratchDoubles = 1 << 19;
// reverse steps on records whose link gradient terms are added in one pass
constexpr int kAkBatch = 8;

// per cut link: the Eq. (213) coefficients, computed in double on the host
// and stored in the precision of the populations (an FP32 handle combines
// them in double all the same)
template <class T>
struct LinkCoefT {
    T c1, c2, c3;        // on f_ibar(x_f,t), f'_i(x_f,t), f'_ibar(x_f,t)
    T wall;              // c4 * 3 w_i rho0 e_i.phi
};
using LinkCoef = LinkCoefT<double>;

struct LinkDeriv {       // d/dgamma of c1, c2, c3 and of the wall term
    double d1, d2, d3, dwall;
};

struct Snapshot {
    void* f = nullptr;
    void* wa = nullptr;
};

// What a recording forward step from the state at t keeps for a reverse
// sweep that does not read the state itself: u(x, t) of the pulled state (D
// planes of stride S, NaN at solid nodes) and, per cut link k = (y, i) in
// sorted order, the forward values of its gradient: f_ibar(y, t) as pulled,
// f'_i(y, t) and f'_ibar(y, t) after the collision.  One record is one
// allocation of record_values() values of the handle's precision: the u
// planes, then the three link runs of max(L, 1) values each.
template <class T>
struct StepRecord {
    T* u;
    T* fib;
    T* fpi;
    T* fpib;
};

struct Engine {
    // configuration
    int lattice = 0, precision = 0, Q = 0, D = 0;
    int device = 0;          // HIP device current at lbm_create
    int64_t nx = 0, ny = 0, nz = 0, N = 0;
    int64_t S = 0;           // N rounded up to whole population blocks (velocity-plane stride)
    int graph_steps = 0;     // >0: replay captured graphs of this many steps
    bool poison = false;     // LBM_DEBUG: outputs filled with NaN before each step
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};   // by starting buffer
    double s[19] = {0};
    double rho0 = 1.0;
    double g[3] = {0, 0, 0};
    int l_rule = 6;
    double b = 1.0;
    int xbc = 0;
    double drho = 0.0;
    size_t elem = 8;         // bytes per stored value

    // geometry
    bool has_geometry = false;
    int64_t n_links = 0, n_fluid = 0;
    int n_tags = 0;
    std::vector<int64_t> perm;          // sorted link k -> caller index
    std::vector<int64_t> lk_node_h;     // sorted
    std::vector<int8_t> lk_dir_h;
    std::vector<double> q_h, wall_u_h;  // sorted, wall_u (L, D)
    std::vector<int32_t> tag_h;

    uint32_t* d_info = nullptr;         // per node: bit 31 solid, bits 19..30 link offset
                                        // within the wave, bits 0..Q-1 link directions
    uint2* d_wave = nullptr;            // per 64-node wave of a node launch: kind, first link
    uint4* d_wact = nullptr;            // the adjoint's non-idle waves in memory order:
    int64_t n_wact = 0;                 // {id, kind | links << 2, first link, 0}
    uint8_t* d_lkdir = nullptr;
    int32_t* d_lknode = nullptr;
    int32_t* d_perm = nullptr;          // sorted link k -> caller index
    int32_t* d_lktag = nullptr;
    LinkCoefT<double>* d_lkcoef = nullptr;   // FP64 handles
    LinkCoefT<float>* d_lkcoef_f = nullptr;  // FP32 handles
    LinkDeriv* d_lkderiv = nullptr;
    double* d_lkc4 = nullptr;           // c4 per link (for dJ/dphi)
    bool two_node = false;              // Eq. (211) instead of Eq. (210)
    double wall_decay = 1.0;            // wall data phi(t) = phi(0) * wall_decay^t
    double wall_scale = 1.0;            // wall_decay^t of the step being launched
    std::vector<uint8_t> ibar_is_link;  // sorted link k: (x_f, ibar) is a link too
    double* d_lkc1d = nullptr;          // c1 applied at the next pull (Eq. (211)), else 0
    double* d_lkd1d = nullptr;          // its gamma derivative

    // state: post-collision array A and link slots of the current time
    Snapshot buf[2];
    int cur = 0;
    bool initialized = false;
    int64_t t = 0;
    bool stepped = false;               // at least one step since init

    // objective
    int obj_kind = 0;
    int obj_tag = 0;
    int64_t obj_t0 = 0, obj_t1 = 0;
    int64_t obj_x_in = 0, obj_x_out = -1;   // pressure-drop planes (-1: nx - 1)
    double obj_a_in = 0.0, obj_a_out = 0.0; // 1 / (fluid nodes of each plane)
    std::vector<int64_t> fluid_per_x;       // fluid nodes of each plane x = const
    double* d_obj_acc = nullptr;        // per-block partial sums
    int64_t obj_acc_len = 0;

    // checkpointed run and adjoint
    std::vector<Snapshot> ckpt;         // snapshot j holds the state at t_run0 + j*every
    std::vector<Snapshot> pool;         // replay pool: every + 1 states, or two
                                        // (ping-pong) when the sweep reads records
    int64_t run_t0 = -1, run_n = 0, run_every = 0;
    void* lam[2] = {nullptr, nullptr};  // adjoint arrays (Q*N values of T)
    // With the rate gradients off the reverse sweep reads step records
    // (StepRecord) instead of the forward states:
    // the checkpointed run records the last step of every segment, the
    // replay of a segment the others.  With a segment of one step the run
    // records every step and keeps no snapshot.
    bool run_urec = false;              // the last run recorded rec_last
    bool run_two_node = false;          // the last run used Eq. (211)
    bool adj_um = false;                // the current sweep reads records
    // Eq. (211) on records: f_ibar(x_f, .) of every link at the run's final
    // state, and at the first step of the segment after the one being
    // reversed (kept before the replay pool is overwritten); L values each
    void* fib_final = nullptr;
    void* fib_next = nullptr;
    std::vector<void*> rec_last;        // per segment: record of its last step
    std::vector<void*> rec_pool;        // per replayed step r of a segment
    double* d_gq = nullptr;             // per link: sum of a_k (dc1 f_ibar + dc2 f'_i + dc3 f'_ibar)
    double* d_gs = nullptr;             // per link: sum of a_k ws (the wall-data terms' factor);
                                        // d_gq + max(L, 1), same allocation
    // reverse steps on records store a_k of every link (one run of max(L, 1)
    // doubles per step, kAkBatch runs) and the terms of the pending steps
    // are added to gq, gs in one pass, step by step in the order taken
    double* ak_buf = nullptr;
    // Eq. (211) on records: the pre-pass's gq term of each pending step
    // (same layout), added just before that step's own terms
    double* tq_buf = nullptr;
    int ak_pending = 0;
    const void* ak_rec[kAkBatch] = {};  // the pending steps' records
    double ak_ws[kAkBatch] = {};        // and their wall-data factors
    double* d_gglob = nullptr;          // per-block partials of dJ/dg (D) and dJ/ds (Q)
    int64_t gglob_len = 0;
    bool have_grad = false;
    // reverse sweep in progress: next step to reverse (relative to the run's
    // first step), segment held by the replay pool
    bool adj_started = false;
    int64_t adj_next = -1;
    int64_t adj_seg = -1;
    int64_t gq_len = 0;
    bool want_ds = true;                // accumulate dJ/ds in the adjoint

    // scratch for reductions and host transfers
    double* d_scratch = nullptr;
    int64_t scratch_len = 0;

    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = -1.0;
    int64_t timed_steps = 0;

    std::string err;
};

// Values (of the handle's precision) of one step record.
inline int64_t record_values(const Engine& e) {
    return (int64_t)e.D * e.S + 3 * (e.n_links > 0 ? e.n_links : 1);
}
// the coefficient table of a handle of precision T
template <class T>
const LinkCoefT<T>* coef_table(const Engine& e) {
    if constexpr (sizeof(T) == 4)
        return e.d_lkcoef_f;
    else
        return e.d_lkcoef;
}

template <class T>
StepRecord<T> record_at(const Engine& e, const void* rec) {
    T* base = (T*)rec;
    const int64_t L1 = e.n_links > 0 ? e.n_links : 1;
    StepRecord<T> r;
    r.u = base;
    r.fib = base + (int64_t)e.D * e.S;
    r.fpi = r.fib + L1;
    r.fpib = r.fpi + L1;
    return r;
}

// ---- launchers (forward.hip) -------------------------------------------------
// Objective terms a step accumulates (per-block sums in double, one thread
// per node): MEAN_UX adds w u_x(x, t); PRESSURE_DROP adds
// w (a_in [x = x_in] - a_out [x = x_out]) (rho(x, t) - rho0).
struct StepObjective {
    double* acc = nullptr;       // per-block accumulator, or null (no objective term)
    double w = 0.0;              // weight of this step's term
    int kind = 0;                // LBM_OBJ_MEAN_UX or LBM_OBJ_PRESSURE_DROP
    uint32_t x_in = 0, x_out = 0;
    double a_in = 0.0, a_out = 0.0;
};

// rec (optional): a step record (StepRecord) receiving u(x, t) of the
// pulled state and the link values of this step
hipError_t launch_step(Engine& e, const Snapshot& in, const Snapshot& out,
                       const StepObjective& obj, void* rec = nullptr);
// initial state: df (Q*N, deviation) or fields rho (N), u (N*D); device pointers
hipError_t launch_init(Engine& e, const double* df, const double* rho,
                       const double* u, const Snapshot& out);
// outputs from the pulled state: rho (N) and u (N*D), or df (Q*N); device
hipError_t launch_observe(Engine& e, const Snapshot& in, double* rho, double* u,
                          double* df);
// per-block partial sums of (drho, rho0 u) over fluid nodes: (nblocks, 1 + D)
hipError_t launch_mass(Engine& e, const Snapshot& in, double* partials,
                       int64_t* nblocks);
// per-block partial sums of a_p (rho - rho0) over the fluid nodes of the
// planes x = x_in (a_in) and x = x_out (a_out); one thread per node of the
// two planes
hipError_t launch_plane_density(Engine& e, const Snapshot& in, uint32_t x_in, uint32_t x_out,
                                double a_in, double a_out, double* partials, int64_t* nblocks);
// per-block partial momentum-exchange force: (nblocks, n_tags, D)
hipError_t launch_force(Engine& e, const Snapshot& post, double* partials,
                        int64_t* nblocks);
// accumulate the x force on one tag into per-block accumulators
hipError_t launch_force_objective(Engine& e, const Snapshot& post, double* acc,
                                  int tag, double weight);
// LBM_DEBUG: fill n values of T (the handle's precision) at p with NaN
hipError_t launch_fill_nan(Engine& e, void* p, size_t n);
// out[c] = sum_b partials[b*cols + c], deterministic
hipError_t launch_sum_blocks(Engine& e, const double* partials, int64_t rows,
                             int64_t cols, double* out);
// device address of the fixed scratch (kNoAllocScratchDoubles doubles) on
// `device`, looked up once per device; shared by every caller on that device
hipError_t noalloc_scratch(int device, double** out);
int64_t step_blocks(const Engine& e);       // logical blocks of a node launch
int64_t adjoint_blocks(const Engine& e);    // blocks of the two adjoint launches together
int64_t link_blocks(const Engine& e);       // blocks of a link launch

// ---- launchers (adjoint.hip) -------------------------------------------------
// One reverse step: lam_in = lambda(t+1) -> lam_out = lambda(t), with the
// forward state at t in `fwd`.  Accumulates per-link and global gradients.
struct AdjointObjective {
    int kind = 0;
    int tag = 0;
    double weight = 0.0;         // 0 when step t is outside the window
    double inv_nfluid = 0.0;
    uint32_t x_in = 0, x_out = 0;        // pressure-drop planes
    double a_in = 0.0, a_out = 0.0;      // 1 / (fluid nodes of each plane)
};
// One reverse step: lambda(t) from lambda(t+1) with the forward states at t
// (`fwd`) and t+1 (`next`), accumulating the gradients.  rec: the record of
// forward step t (rate gradients off; fwd and next are
// then not read and may be null), or null to read the states.  With a
// record the link gradient terms of the step stay pending (the record must
// live until launch_link_sums); kAkBatch pending steps are summed at once.
hipError_t launch_adjoint_step(Engine& e, const Snapshot* fwd, const Snapshot* next,
                               const void* rec, const void* lam_in, void* lam_out,
                               const AdjointObjective& obj);
// the pending steps' link gradient terms into gq, gs (no-op if none pend)
hipError_t launch_link_sums(Engine& e);
hipError_t launch_adjoint_out(Engine& e, const void* lam, double* out);
// per-link gradients from the sweep's sums, in the caller's link order, into
// device buffers: dq (L doubles) and dphi (L*D, link-major); either may be
// null
hipError_t launch_link_gradients(Engine& e, double* dq, double* dphi);
// Eq. (211) links: move c1 * (adjoint of f_i(x_f, t+1)) onto the adjoint of
// f_ibar(x_f, t+1) and add the gamma-derivative of that term, with
// f_ibar(x_f, t+1) pulled from the forward state at t+1 (`next`) or read
// from fib_next (L values of T: the link run of the record of step t+1);
// exactly one of the two is given.  With fib_next (a sweep on records) the
// gamma-derivative term stays pending with the step that launch_adjoint_step
// takes next.
hipError_t launch_two_node_adjoint(Engine& e, const Snapshot* next, const void* fib_next,
                                   void* lam_in, const AdjointObjective& obj);
// out[k] = f_ibar(x_f, t) as the pull of the opposite direction at link k's
// node reads it from the state s (L values of T)
hipError_t launch_link_pull(Engine& e, const Snapshot& s, void* out);

}  // namespace lbe
