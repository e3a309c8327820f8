// Host-only driver for the engine's geometry tables (csrc/geometry.cpp),
// built with the address and undefined-behaviour sanitizers by
// tests/test_host_sanitize.py.  It feeds seeded random geometries, valid
// and invalid, and checks the error codes and the invariants of the tables;
// any out-of-bounds access or undefined operation aborts the run.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "../../paper_1712_08288_amd/csrc/geometry.hpp"

namespace {

const int E2[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                      {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
const int E3[19][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                       {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, 1, 0}, {1, -1, 0},
                       {-1, -1, 0}, {1, 0, 1},   {-1, 0, 1}, {1, 0, -1}, {-1, 0, -1},
                       {0, 1, 1},   {0, -1, 1},  {0, 1, -1}, {0, -1, -1}};

int failures = 0;

void check(bool ok, const std::string& what) {
    if (!ok) {
        std::printf("FAIL: %s\n", what.c_str());
        ++failures;
    }
}

struct Case {
    lbe::GeomDomain d;
    std::vector<uint8_t> solid;
    std::vector<int64_t> node;
    std::vector<int8_t> dir;
    std::vector<double> q, wall_u;
    std::vector<int32_t> tag;
};

// x - e_i with y, z periodic and x periodic or clamped (written here
// independently of the unit under test)
int64_t source(const lbe::GeomDomain& d, int64_t n, int i) {
    const int64_t x = n % d.nx, y = (n / d.nx) % d.ny, z = n / (d.nx * d.ny);
    int64_t sx = x - d.e[i][0];
    if (d.outflow) sx = sx < 0 ? 0 : (sx >= d.nx ? d.nx - 1 : sx);
    else sx = (sx + d.nx) % d.nx;
    const int64_t sy = (y - d.e[i][1] + d.ny) % d.ny;
    const int64_t sz = (z - d.e[i][2] + d.nz) % d.nz;
    return sx + d.nx * (sy + d.ny * sz);
}

Case make(std::mt19937_64& rng, bool three_d, int64_t nx, int64_t ny, int64_t nz, bool outflow,
          double fill) {
    Case c;
    c.d.Q = three_d ? 19 : 9;
    c.d.D = three_d ? 3 : 2;
    c.d.e = three_d ? E3 : E2;
    c.d.nx = nx;
    c.d.ny = ny;
    c.d.nz = three_d ? nz : 1;
    c.d.outflow = outflow;
    const int64_t N = c.d.nx * c.d.ny * c.d.nz;
    std::uniform_real_distribution<double> u(0.0, 1.0);
    c.solid.assign(N, 0);
    for (int64_t n = 0; n < N; ++n) {
        c.solid[n] = u(rng) < fill ? 1 : 0;
        if (outflow && n % nx == 0) c.solid[n] = 1;
    }
    for (int64_t n = 0; n < N; ++n) {
        if (c.solid[n]) continue;
        for (int i = 1; i < c.d.Q; ++i)
            if (c.solid[source(c.d, n, i)]) {
                c.node.push_back(n);
                c.dir.push_back((int8_t)i);
                c.q.push_back(1e-3 + 0.999 * u(rng));
                for (int a = 0; a < c.d.D; ++a) c.wall_u.push_back(0.01 * (u(rng) - 0.5));
                c.tag.push_back((int32_t)(u(rng) * 3));
            }
    }
    // hand the links over in a shuffled order (the unit sorts them)
    std::vector<size_t> p(c.node.size());
    for (size_t k = 0; k < p.size(); ++k) p[k] = k;
    std::shuffle(p.begin(), p.end(), rng);
    Case s = c;
    for (size_t k = 0; k < p.size(); ++k) {
        s.node[k] = c.node[p[k]];
        s.dir[k] = c.dir[p[k]];
        s.q[k] = c.q[p[k]];
        s.tag[k] = c.tag[p[k]];
        for (int a = 0; a < c.d.D; ++a) s.wall_u[k * c.d.D + a] = c.wall_u[p[k] * c.d.D + a];
    }
    return s;
}

int run(const Case& c, lbe::GeomTables& t, std::string& err) {
    lbe::GeomLinks l;
    l.n = (int64_t)c.node.size();
    l.node = c.node.data();
    l.dir = c.dir.data();
    l.q = c.q.data();
    l.wall_u = c.wall_u.empty() ? nullptr : c.wall_u.data();
    l.tag = c.tag.data();
    return lbe::build_geometry(c.d, c.solid.data(), l, t, err);
}

void check_tables(const Case& c, const lbe::GeomTables& t, const std::string& name) {
    const int64_t N = c.d.nx * c.d.ny * c.d.nz, L = (int64_t)c.node.size();
    check((int64_t)t.perm.size() == L && (int64_t)t.node.size() == L, name + ": sizes");
    std::vector<int> seen(L, 0);
    for (int64_t k = 0; k < L; ++k) {
        check(t.perm[k] >= 0 && t.perm[k] < L, name + ": perm range");
        if (t.perm[k] >= 0 && t.perm[k] < L) ++seen[t.perm[k]];
        if (k > 0)
            check(t.node[k - 1] < t.node[k] || (t.node[k - 1] == t.node[k] && t.dir[k - 1] < t.dir[k]),
                  name + ": sorted");
        check(t.node[k] == c.node[t.perm[k]] && t.dir[k] == c.dir[t.perm[k]], name + ": permuted copy");
    }
    for (int64_t k = 0; k < L; ++k) check(seen[k] == 1, name + ": perm is a permutation");
    int64_t fluid = 0, links_in_waves = 0, nonidle = 0;
    for (int64_t n = 0; n < N; ++n) fluid += c.solid[n] ? 0 : 1;
    check(fluid == t.n_fluid, name + ": fluid count");
    for (size_t w = 0; w < t.wave.size(); ++w) {
        const uint32_t kind = t.wave[w].x & 3u, cnt = (t.wave[w].x >> 2) & 0x3FFFu;
        check(kind <= 2u, name + ": wave kind");
        check((int64_t)t.wave[w].y == links_in_waves, name + ": first link of a wave");
        links_in_waves += cnt;
        nonidle += kind != 2u;
        // a node's first link is its wave's first link plus its offset
        for (int64_t n = (int64_t)w * c.d.wave; n < std::min<int64_t>(N, (int64_t)(w + 1) * c.d.wave); ++n) {
            if (c.solid[n]) {
                check(t.info[n] == 0x80000000u, name + ": solid info word");
                continue;
            }
            const uint32_t m = t.info[n] & ((1u << 19) - 1u);
            if (!m) continue;
            const int64_t first = t.wave[w].y + ((t.info[n] >> 19) & 0xFFFu);
            check(first >= 0 && first < L && t.node[first] == n, name + ": node's first link");
        }
    }
    check(links_in_waves == L, name + ": links over waves");
    check((int64_t)t.wact.size() == nonidle, name + ": active wave list");
}

void expect(const Case& c, int code, const std::string& name) {
    lbe::GeomTables t;
    std::string err;
    const int rc = run(c, t, err);
    check(rc == code, name + ": expected " + std::to_string(code) + ", got " + std::to_string(rc) +
                          " (" + err + ")");
    if (code == 0 && rc == 0) check_tables(c, t, name);
}

}  // namespace

int main() {
    std::mt19937_64 rng(12345);
    int n_valid = 0;
    struct Shape { bool d3; int64_t nx, ny, nz; bool outflow; double fill; };
    const Shape shapes[] = {{false, 37, 23, 1, false, 0.15}, {false, 64, 8, 1, false, 0.3},
                            {false, 5, 3, 1, false, 0.2},    {false, 29, 17, 1, true, 0.1},
                            {true, 13, 11, 9, false, 0.12},  {true, 16, 8, 4, true, 0.2},
                            {true, 3, 3, 3, false, 0.3},     {false, 300, 7, 1, false, 0.05},
                            {false, 12, 10, 1, false, 0.0},  {true, 7, 5, 4, false, 1.0}};
    for (int rep = 0; rep < 4; ++rep)
        for (const Shape& s : shapes) {
            const Case c = make(rng, s.d3, s.nx, s.ny, s.nz, s.outflow, s.fill);
            const std::string name = std::string(s.d3 ? "3d " : "2d ") + std::to_string(s.nx) + "x" +
                                     std::to_string(s.ny) + "x" + std::to_string(s.nz);
            expect(c, 0, name);
            ++n_valid;
            if (c.node.empty()) continue;
            Case bad = c;
            bad.node.push_back(bad.node[0]);         // duplicate link
            bad.dir.push_back(bad.dir[0]);
            bad.q.push_back(0.5);
            for (int a = 0; a < c.d.D; ++a) bad.wall_u.push_back(0.0);
            bad.tag.push_back(0);
            expect(bad, LBM_EGEOM, name + " duplicate");
            bad = c;                                 // missing link
            bad.node.pop_back();
            bad.dir.pop_back();
            bad.q.pop_back();
            bad.tag.pop_back();
            for (int a = 0; a < c.d.D; ++a) bad.wall_u.pop_back();
            expect(bad, LBM_EGEOM, name + " missing");
            bad = c;
            bad.q[0] = 0.0;
            expect(bad, LBM_EINVAL, name + " q = 0");
            bad = c;
            bad.q[0] = std::nan("");
            expect(bad, LBM_EINVAL, name + " q NaN");
            bad = c;
            bad.dir[0] = (int8_t)c.d.Q;
            expect(bad, LBM_EINVAL, name + " direction out of range");
            bad = c;
            bad.dir[0] = -3;
            expect(bad, LBM_EINVAL, name + " negative direction");
            bad = c;
            bad.node[0] = c.d.nx * c.d.ny * c.d.nz;
            expect(bad, LBM_EINVAL, name + " node out of range");
            bad = c;
            bad.tag[0] = -1;
            expect(bad, LBM_EINVAL, name + " negative tag");
            bad = c;
            bad.wall_u[0] = INFINITY;
            expect(bad, LBM_EINVAL, name + " wall velocity");
            bad = c;
            bad.solid[bad.node[0]] = 1;
            expect(bad, LBM_EGEOM, name + " link at a solid node");
            bad = c;
            bad.solid[0] = 2;
            expect(bad, LBM_EINVAL, name + " solid value");
        }
    // outflow with a fluid node at x = 0
    Case c = make(rng, false, 20, 9, 1, true, 0.1);
    c.solid[c.d.nx * 3] = 0;
    expect(c, LBM_EGEOM, "outflow fluid at x = 0");
    std::printf("%s: %d valid geometries, %d failures\n", failures ? "FAILED" : "ok", n_valid,
                failures);
    return failures ? 1 : 0;
}
