// RWG bases of a planar element and their EFIE interaction blocks (internal).
#pragma once

#include <vector>

#include "../../include/mbt.h"
#include "common.h"

namespace mbt {

constexpr int kRwgQ = 7;          // points of the triangle rule
constexpr int kRwgMaxTri = 256;   // triangles per element

// Host description of one element's RWG functions, in the element frame.
struct RwgMesh {
    int nt = 0, M = 0;
    std::vector<double2> qp;     // nt * kRwgQ rule points
    std::vector<double> qw;      // nt * kRwgQ rule weights times the triangle area
    std::vector<double2> tv;     // nt * 3 vertices
    std::vector<double> area;    // nt
    std::vector<int> btri;       // 2M: T+ and T- of each basis
    std::vector<double2> bfree;  // 2M: the vertex of T+ / T- opposite the basis edge
    std::vector<double> blen;    // M: edge length
    PortDef port;                // gap bases and weights sign * length
};

// Bases of a mesh (interior edges in increasing vertex-pair order; T+ is the
// lower-index triangle); throws Error(-1) on an invalid mesh.
RwgMesh rwg_from_mesh(const mbt_rwg_mesh& mesh);

// T[(dy+ny-1)*nox + (dx+nx-1)][p][q]: Galerkin EFIE block between test basis p
// of the element at lattice offset d from the source element and source basis q,
// at wavenumber k (1/wavelength units of the mesh).
void rwg_fill_blocks(const Geom& g, const RwgMesh& mesh, double k, double2* T, hipStream_t s);

}  // namespace mbt
