// Host-side geometry tables (see geometry.hpp).
#include "geometry.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

#include "../../include/lbm.h"

namespace lbe {

int64_t pull_source(const GeomDomain& d, int64_t x, int64_t y, int64_t z, int i) {
    int64_t sx = x - d.e[i][0];
    const int64_t sy = ((y - d.e[i][1]) % d.ny + d.ny) % d.ny;
    const int64_t sz = ((z - (d.D == 3 ? d.e[i][2] : 0)) % d.nz + d.nz) % d.nz;
    if (d.outflow) {
        if (sx >= d.nx) sx = d.nx - 1;
        if (sx < 0) sx = 0;
    } else {
        sx = (sx % d.nx + d.nx) % d.nx;
    }
    return sx + d.nx * (sy + d.ny * sz);
}

int build_geometry(const GeomDomain& d, const uint8_t* solid, const GeomLinks& lk,
                   GeomTables& out, std::string& err) {
    const int64_t N = d.nx * d.ny * d.nz;
    const int Q = d.Q, D = d.D;
    const int64_t L = lk.n;
    auto fail = [&](int code, const char* msg) {
        err = msg;
        return code;
    };
    if (!solid) return fail(LBM_EINVAL, "solid mask is NULL");
    if (L < 0 || L >= (1LL << 26)) return fail(LBM_EINVAL, "number of links out of range [0, 2^26)");
    if (L > 0 && (!lk.node || !lk.dir || !lk.q)) return fail(LBM_EINVAL, "link arrays are NULL");
    for (int64_t n = 0; n < N; ++n)
        if (solid[n] > 1) return fail(LBM_EINVAL, "solid mask values must be 0 or 1");
    for (int64_t k = 0; k < L; ++k) {
        if (lk.node[k] < 0 || lk.node[k] >= N) return fail(LBM_EINVAL, "link node out of range");
        if (lk.dir[k] < 1 || lk.dir[k] >= Q) return fail(LBM_EINVAL, "link direction out of range");
        if (!(lk.q[k] > 0.0 && lk.q[k] <= 1.0)) return fail(LBM_EINVAL, "q must lie in (0, 1]");
        if (solid[lk.node[k]]) return fail(LBM_EGEOM, "link at a solid node");
        if (lk.tag && lk.tag[k] < 0) return fail(LBM_EINVAL, "negative tag");
        if (lk.wall_u)
            for (int a = 0; a < D; ++a)
                if (!std::isfinite(lk.wall_u[k * D + a]))
                    return fail(LBM_EINVAL, "wall velocity not finite");
    }
    // sort by (node, dir)
    std::vector<int64_t> perm(L);
    std::iota(perm.begin(), perm.end(), 0);
    std::sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) {
        return lk.node[a] != lk.node[b] ? lk.node[a] < lk.node[b] : lk.dir[a] < lk.dir[b];
    });
    // per-node link mask, duplicates, consistency with the mask
    std::vector<uint32_t> mask(N, 0u);
    for (int64_t k = 0; k < L; ++k) {
        const uint32_t bit = 1u << lk.dir[k];
        if (mask[lk.node[k]] & bit) return fail(LBM_EGEOM, "duplicate cut link");
        mask[lk.node[k]] |= bit;
    }
    int64_t n_fluid = 0;
    std::vector<int64_t> fluid_per_x(d.nx, 0);
    for (int64_t z = 0; z < d.nz; ++z)
        for (int64_t y = 0; y < d.ny; ++y)
            for (int64_t x = 0; x < d.nx; ++x) {
                const int64_t n = x + d.nx * (y + d.ny * z);
                if (solid[n]) continue;
                ++n_fluid;
                ++fluid_per_x[x];
                if (d.outflow && x == 0)
                    return fail(LBM_EGEOM, "outflow x boundary needs a solid column x = 0");
                for (int i = 1; i < Q; ++i) {
                    const bool need = solid[pull_source(d, x, y, z, i)] != 0;
                    const bool have = (mask[n] >> i) & 1u;
                    if (need != have)
                        return fail(LBM_EGEOM,
                                    need ? "fluid node pulls from a solid node without a cut link"
                                         : "cut link whose pull source is fluid");
                }
            }
    // host copies in sorted order
    out.perm = perm;
    out.n_fluid = n_fluid;
    out.fluid_per_x = fluid_per_x;
    out.node.resize(L);
    out.dir.resize(L);
    out.q.resize(L);
    out.wall_u.assign((size_t)L * D, 0.0);
    out.tag.resize(L);
    int max_tag = -1;
    for (int64_t k = 0; k < L; ++k) {
        const int64_t p = perm[k];
        out.node[k] = lk.node[p];
        out.dir[k] = lk.dir[p];
        out.q[k] = lk.q[p];
        if (lk.wall_u)
            for (int a = 0; a < D; ++a) out.wall_u[k * D + a] = lk.wall_u[p * D + a];
        out.tag[k] = lk.tag ? lk.tag[p] : 0;
        max_tag = std::max(max_tag, out.tag[k]);
    }
    out.n_tags = max_tag + 1;
    out.ibar_is_link.assign(L, 0);
    for (int64_t k = 0; k < L; ++k) {
        const int i = out.dir[k];
        int ib = 0;
        for (int j = 0; j < Q; ++j) {
            bool opp = true;
            for (int a = 0; a < 3; ++a) opp = opp && d.e[j][a] == -d.e[i][a];
            if (opp) ib = j;
        }
        const int64_t y = out.node[k];
        out.ibar_is_link[k] = (mask[y] >> ib) & 1u;
    }
    // per node: bit 31 solid, else the link-direction mask and, in bits
    // 19..30, the number of links at earlier nodes of its wave; per wave of a
    // node launch (wave consecutive node indices): its kind -- idle (no
    // fluid), plain (every node fluid without links) or mixed -- with its link
    // count, the eighths of its lanes without a fluid node, and the index of
    // its first link (links are sorted by node)
    out.info.assign(N, 0u);
    const int64_t W = d.wave;
    const int64_t nwave = (N + d.block - 1) / d.block * (d.block / W);
    out.wave.assign(nwave, WaveWord{2u, 0u});
    int64_t k = 0;
    for (int64_t w = 0; w < nwave; ++w) {
        const int64_t n0 = w * W;
        const int64_t nin = std::max<int64_t>(0, std::min<int64_t>(W, N - n0));
        bool any_fluid = false, all_plain = nin == W;
        const int64_t k0 = k;
        for (int64_t n = n0; n < n0 + nin; ++n) {
            if (solid[n]) {
                out.info[n] = 0x80000000u;
                all_plain = false;
                continue;
            }
            any_fluid = true;
            all_plain = all_plain && mask[n] == 0u;
            out.info[n] = mask[n] | ((uint32_t)(k - k0) << 19);
            k += __builtin_popcount(mask[n]);
        }
        const uint32_t kind = !any_fluid ? 2u : (all_plain ? 1u : 0u);
        uint32_t dead = 0u;   // eighths of W / 8 lanes without a fluid node
        const int64_t e8 = W / 8;
        for (int qd = 0; qd < 8; ++qd) {
            bool fluid = false;
            for (int64_t n = n0 + e8 * qd; n < std::min<int64_t>(n0 + e8 * qd + e8, N); ++n)
                fluid = fluid || !solid[n];
            if (!fluid) dead |= 1u << qd;
        }
        if (kind != 0u) dead = 0u;
        out.wave[w] = WaveWord{kind | ((uint32_t)(k - k0) << 2) | (dead << 16), (uint32_t)k0};
    }
    if (k != L) return fail(LBM_EGEOM, "link count mismatch");
    out.wact.clear();
    for (size_t w = 0; w < out.wave.size(); ++w)
        if ((out.wave[w].x & 3u) != 2u)
            out.wact.push_back(WaveEntry{(uint32_t)w, out.wave[w].x, out.wave[w].y, 0u});
    return 0;
}

}  // namespace lbe
