// Internal interfaces between the host-side translation units of libinrf.
#pragma once

#include <cstdint>
#include <vector>

#include "inrf.h"

namespace inrf {

// Occupied vertices of one level as ascending linear keys (z*(N+1)+y)*(N+1)+x.
std::vector<int64_t> shell_keys(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, int N,
                                int dilate, int threads);

struct PshLevel {
    int32_t res = 0, mbar = 0, rbar = 0, restarts = 0;
    std::vector<int64_t> keys;   // ascending linear keys
    std::vector<uint32_t> phi;   // packed offsets, rbar^3
    std::vector<int32_t> slots;  // slot of each key
};

// Offset table and key->slot map of one level (throws inrf::Error).
void build_psh_level(PshLevel& L, const inrf_psh_params& p);

}  // namespace inrf

struct inrf_psh {
    std::vector<inrf::PshLevel> levels;
};
