// lst_internal.h -- structures shared by the host geometry builder and the
// device engine of liblst (library-internal, not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "lst.h"

namespace lst {

// Per-module mini-doublet window constants (binary32, rounded once from
// binary64).  Barrel: S = sin(max azimuth change between the sensors), G =
// gap / cos(turning angle at the upper sensor), K = z resolution term.
// Endcap: S as above, D = largest radial change between the sensors + r
// resolution term.
struct MdConst {
    float S, G, K, D;
};

// Line-segment window constants of one class of module pairs (A -> B).
//   type 0: barrel -> barrel, 1: endcap -> endcap, 2: barrel -> endcap.
struct LsClass {
    float S;                 // sin(max azimuth change between the anchors)
    float rho_lo, rho_hi;    // BB: arc-length ratio s(r_B)/s(r_A) range
    float lam_lo, lam_hi;    // BB: segment / mini-doublet bend ratio range
    float tau;               // BB: bend resolution term
    float lo_fac, hi_fac;    // EE: r_B / r_A range factors
    float cf;                // BE: chord/arc factor at the outer ring edge
    float zs;                // BE: side of the disk (+1 / -1)
    float zbpl, zbml;        // BE: |z_B| + L, |z_B| - L
    uint32_t type;
    uint32_t pad[3];
};
static_assert(sizeof(LsClass) == 64, "LsClass layout");

// Largest azimuth difference of a segment's anchors for a class, asin(S),
// with room for the binary32 arithmetic of the per-segment reach test.
float ls_reach(const LsClass &k);

// Surfaces (barrel layers, disks) as seen by the seed lookup.
struct Surface {
    uint32_t kind;           // LST_BARREL / LST_ENDCAP
    int32_t side;
    float r1, r2;            // anchor radius range (padded)
    float z1, z2;            // barrel: z extent (padded); endcap: plane z of the lower sensor (z1 == z2)
    float pad[2];
};

// Scalars used by the cuts (binary32) and by the seed cuts (binary64).
struct Consts {
    float L, ec, kmaxf, khalf, ns, srp, sc, Kb;
    double B, n_sigma, sig_rphi, sig_c, kB;
    uint32_t n_mod, n_surf, flags, nphi;
    uint32_t nkb;            // curvature bins of the seed-lookup buckets (per resolution class)
    float kspan;             // curvature bins cover [-kspan, kspan]
    float sk_cls[3];         // resolution classes: sigma_kappa <= sk_cls[i]; larger ones go to the wide bin
    uint32_t ls_group;       // segment walk: runs of edges per group (4, 6, 8)
    uint32_t ls_waves;       // segment walk: minimum waves per SIMD (0: the compiler's choice, 6, 8)
};

struct Geometry {
    uint32_t n_mod = 0;
    uint32_t nb = 0, nd = 0;         // barrel layers, disks per side
    std::vector<uint32_t> kind;      // per module
    std::vector<uint32_t> surf;      // per module surface id
    std::vector<MdConst> mdc;        // per module
    std::vector<uint32_t> edge_begin; // n_mod + 1
    std::vector<uint32_t> edge_dst;   // per edge: destination module
    std::vector<uint32_t> edge_cls;   // per edge: class id
    std::vector<LsClass> classes;
    // segment-walk runs: edges of a module to consecutive destinations of
    // one class with evenly spaced azimuth centres, one record per run
    // (first destination, class | length << 24, azimuth centre of the first
    // module, 1 / pitch) and its window (radians for a run of one module,
    // module indices otherwise)
    std::vector<uint32_t> run_begin;  // n_mod + 1
    std::vector<uint32_t> run_rec;    // 4 per run
    std::vector<float> run_win;       // per run
    // per module: azimuth centre in (-pi, pi] and half-width, widened by the
    // connection map's hit-position margin (radians)
    std::vector<float> mod_phi;
    // per module, 8 floats: the extent the ingest check accepts (azimuth
    // centre, half-width, coarse lo, coarse hi) and the sensor positions
    // (s_lo, s_hi, tolerance, 0)
    std::vector<float> mod_ext;
    std::vector<Surface> surfaces;
    Consts c{};
};

// Builds every host-side table from a validated module list.
lst_status build_geometry(const lst_params &p, const lst_module_desc *m, uint32_t n,
                          Geometry &g, std::string &err);

// As build_geometry, through a cache directory: the tables of a module list
// and parameters are read from dir when a blob built from exactly the same
// inputs is there (from_cache = true), otherwise built and written there
// (a blob that cannot be read or written is ignored: the tables are built).
// dir empty: build_geometry.
lst_status build_geometry_cached(const lst_params &p, const lst_module_desc *m, uint32_t n,
                                 const std::string &dir, Geometry &g, std::string &err, bool &from_cache);

}  // namespace lst
