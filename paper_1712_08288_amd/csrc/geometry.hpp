// Host-side geometry tables of the engine: validation of the solid mask and
// the cut links, the link sort, and the per-node and per-wave tables the
// kernels read.  Plain C++ (no HIP), so that it can also be built and run
// under the host address and undefined-behaviour sanitizers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace lbe {

// What the geometry tables need to know about the lattice and the domain.
struct GeomDomain {
    int Q = 0, D = 0;
    const int (*e)[3] = nullptr;   // e[i][a], a < 3 (z component 0 in 2D)
    int64_t nx = 0, ny = 0, nz = 0;
    bool outflow = false;          // zero-gradient x boundary (clamped x pull)
    int block = 256;               // threads per block of node launches
    int wave = 64;                 // nodes per wave
};

// The caller's cut links (any order), as passed to lbm_set_geometry.
struct GeomLinks {
    int64_t n = 0;
    const int64_t* node = nullptr;
    const int8_t* dir = nullptr;
    const double* q = nullptr;
    const double* wall_u = nullptr;   // n * D values or null (0)
    const int32_t* tag = nullptr;     // or null (0)
};

struct WaveWord {   // same layout as the device's uint2
    uint32_t x, y;
};
struct WaveEntry {  // same layout as the device's uint4
    uint32_t x, y, z, w;
};

struct GeomTables {
    int64_t n_fluid = 0;
    int n_tags = 0;
    std::vector<int64_t> perm;          // sorted link k -> caller index
    std::vector<int64_t> node;          // sorted by (node, dir)
    std::vector<int8_t> dir;
    std::vector<double> q, wall_u;      // wall_u (L, D)
    std::vector<int32_t> tag;
    std::vector<uint8_t> ibar_is_link;  // (x_f, ibar) is a link too
    std::vector<int64_t> fluid_per_x;   // fluid nodes of each plane x = const
    // per node: bit 31 solid; else bits 0..Q-1 the link directions and bits
    // 19..30 the links at earlier nodes of its wave
    std::vector<uint32_t> info;
    // per wave of a node launch: x = kind (0 mixed, 1 plain, 2 idle) | links
    // << 2 | eighths without fluid << 16, y = first link
    std::vector<WaveWord> wave;
    // the non-idle waves in memory order: {wave, wave.x, wave.y, 0}
    std::vector<WaveEntry> wact;
};

// Node index of the pull source of direction i at (x, y, z): periodic in y
// and z, periodic in x or clamped to [0, nx) with the outflow boundary.
int64_t pull_source(const GeomDomain& d, int64_t x, int64_t y, int64_t z, int i);

// Validate and build every table.  Returns 0, or an lbm.h error code
// (LBM_EINVAL, LBM_EGEOM) with the reason in `err`.
int build_geometry(const GeomDomain& d, const uint8_t* solid, const GeomLinks& links,
                   GeomTables& out, std::string& err);

}  // namespace lbe
