// Host-side mesh data of the DG solver (FP64): connectivity, affine geometry,
// multi-rate levels and the TVB neighbour stencil of one triangulation.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "host_refelem.hpp"

namespace dgswe {

struct HostMesh {
    int K = 0, Nv = 0;
    std::vector<double> vx, vy;
    std::vector<int32_t> etov;      // K x 3, counter-clockwise
    std::vector<int32_t> etoe;      // K x 3 (self for a wall face)
    std::vector<int8_t> etof;       // K x 3 (own face for a wall face)
    std::vector<uint8_t> wall;      // K x 3
    std::vector<double> rx, ry, sx, sy, J;   // K
    std::vector<double> nx, ny, sJ, fscale;  // K x 3
    std::vector<double> inradius, dk;        // K (dk = longest edge)
    std::vector<int8_t> level;               // K, 1 = finest
    std::vector<int8_t> pair;                // K x 3 x 2
    std::vector<double> alpha;               // K x 3 x 2
    std::vector<double> dir;                 // K x 3 x 2 unit (m_i - b0)/|m_i - b0|
};

// Returns "" on success, else an error message (malformed mesh).
// bc: optional K x 3 face tags (0 = interior where shared, 1 = wall)
std::string build_host_mesh(int nv, const double* vx, const double* vy, int K,
                            const int32_t* etov, const int8_t* bc, HostMesh& m);
void assign_levels(HostMesh& m, int max_levels);
void build_tvb_stencil(HostMesh& m);
void node_coords(const HostMesh& m, const RefElement& re, double* x, double* y);

}  // namespace dgswe
