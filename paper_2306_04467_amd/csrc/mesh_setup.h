// Host-side mesh preprocessing for the GKS library (FP64, once per mesh).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace gks {

// Structure-of-arrays tables consumed by the device kernels.  "T" = triangles, "E" = edges,
// "NG" = ghost cells (mirror images used by stencils next to walls); cell-indexed state arrays
// on the device have T + NG entries, the ghost part refreshed from its source cell every stage.
struct HostMesh {
    int64_t nt = 0, ne = 0, ng = 0;
    double dxmin = 0;                // smallest cell size (smallest altitude) over the mesh
    // cells
    std::vector<double> area;        // [T]
    std::vector<double> hs;          // [T] length scale sqrt(2 |Omega|) of the scaled coordinates
    std::vector<double> vtx;         // [6][T] vertex offsets from the centroid, divided by hs
    std::vector<double> nbc;         // [6][T] centroid offsets of the 3 face-neighbour images / hs
    std::vector<uint8_t> cand;       // [T] bit s: the plane through the averages of the cell and
                                     // its face neighbours s, s+1 is a candidate of the nonlinear
                                     // reconstruction (its two centroid offsets are not nearly
                                     // parallel)
    std::vector<double> fl;          // [3][T] sigma_k |Gamma_k| / |Omega|
    std::vector<double> gg;          // [6][T] sigma_k |Gamma_k| n_k / |Omega| (x, y per edge)
    std::vector<double> Bbar;        // [T] cell average of the piecewise-linear bottom
    std::vector<double> gB;          // [2][T] its (constant) gradient
    std::vector<int32_t> cedge;      // [3][T] edge of local edge k: e (cell is left) or ~e (right)
    std::vector<int32_t> sten;       // [9][T] stencil cells (face neighbours, then second ring)
    std::vector<double> M;           // [153][T] least-squares operator, row k*17+r
    std::vector<double> igeo;        // [6][T] indicator geometry: area ratios of the 3 face
                                     // neighbours, then the 3 edge lengths over hs
    // edges
    std::vector<int32_t> eL, eR;     // [E] left / right cell, eR = -1 on walls, -2 on free
                                     // (zero-gradient) boundaries
    std::vector<int32_t> eslot;      // [E] local edge index in L | (in R << 2)
    std::vector<double> en;          // [2][E] unit normal from L to R
    std::vector<double> eBgp;        // [2][E] bottom at the two Gauss points (L orientation)
    std::vector<double> egB;         // [2][E] single-valued bottom gradient at the edge
    // ghosts
    std::vector<int32_t> gsrc;       // [NG] source cell
    std::vector<double> gR;          // [8][NG] orthogonal map of the ghost image (applied to
                                     // gradient directions), then the map of momentum vectors
                                     // (the same across walls, the identity across free edges)
    // scenarios (independent meshes concatenated into one); a single mesh has S = 1 and
    // empty cscen / escen
    int32_t S = 1;
    std::vector<int32_t> cscen, escen;  // [T], [E] scenario of each cell / edge
    std::vector<int64_t> scell;         // [S + 1] first cell of each scenario
    std::vector<double> sdxmin;         // [S]
};

// Smallest sine of the angle between the two centroid offsets of a plane candidate.
constexpr double PLANE_SINE_MIN = 0.2;

// Returns 0 on success, otherwise fills err.  bc: 0 walls, 1 periodic on [0,L0]x[0,L1], 2 free
// (zero-gradient) boundaries.
int build_host_mesh(const double *xy, int64_t nn, const int32_t *tri, int64_t nt, const double *B,
                    int bc, const double *L, HostMesh &m, std::string &err);

// Concatenate independent meshes into one with S scenarios (cells, edges and ghosts renumbered
// with offsets; ghost cells of all scenarios follow all real cells).
HostMesh concat_host_meshes(const std::vector<const HostMesh *> &parts);

}  // namespace gks
