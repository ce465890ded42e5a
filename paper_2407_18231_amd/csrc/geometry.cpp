// geometry.cpp -- host side of liblst: validates a module table, derives the
// per-module and per-module-pair window constants (binary64, rounded once to
// binary32) and builds the module connection map ("precomputed connection
// maps for modules", Sec. 1) by an interval test of the line-segment windows
// over each module pair's extents.
//
// Window reading (the paper defers its cuts to its references): every window
// is the closed form of a prompt helix with |curvature| <= kappa_max (the pT
// threshold of Sec. 1) and vertex z within +/- L, widened by n_sigma times
// the hit resolution.  A(r) = asin(r kappa_max / 2) is half the turning angle
// at radius r; s(r) = 2 A(r) / kappa the transverse arc length; f(x) =
// asin(x) / x the arc/chord ratio.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>

#include <unistd.h>

#include "lst_internal.h"

namespace lst {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;

// The connection map and the seed-lookup surfaces cover hits up to this many
// resolutions outside their module's extent (sigma_rphi over the module's
// inner radius in azimuth, sigma_c along z in the barrel and r on a disk).
constexpr double kEdgeSigmas = 6.0;
// Input contract checked at ingest: a hit lies within this many resolutions
// of its module's extent, and on its sensor (barrel radius, disk plane z)
// within kSurfTol.  The half resolution between the two margins absorbs the
// binary32 rounding of the ingest check.
constexpr double kHitSigmas = 5.5;
constexpr double kSurfTol = 0.008;   // cm; the map and the roads allow 0.01

double half_turn(double r, double k)
{
    double x = r * k / 2.0;
    if (x > 1.0) x = 1.0;
    return std::asin(x);
}

double arc_over_chord(double x) { return x == 0.0 ? 1.0 : std::asin(x) / x; }

bool finite(double v) { return std::isfinite(v); }

double wrap2pi(double x)
{
    x = std::fmod(x, kTwoPi);
    if (x < 0) x += kTwoPi;
    return x;
}

// x - 2 pi k in (-pi, pi]
double wrap_pi(double x)
{
    x = wrap2pi(x);
    return x > kPi ? x - kTwoPi : x;
}

// smallest azimuth distance between arcs [a0, a1] and [b0, b1]
double arc_gap(double a0, double a1, double b0, double b1)
{
    if (wrap2pi(b0 - a0) <= a1 - a0 || wrap2pi(a0 - b0) <= b1 - b0) return 0.0;
    return std::min(wrap2pi(b0 - a1), wrap2pi(a0 - b1));
}

struct ZoneKey {
    uint32_t kind;
    double s_lo, s_hi, c_min, c_max;
    bool operator<(const ZoneKey &o) const
    {
        return std::tie(kind, s_lo, s_hi, c_min, c_max) <
               std::tie(o.kind, o.s_lo, o.s_hi, o.c_min, o.c_max);
    }
};

}  // namespace

float ls_reach(const LsClass &k) { return (float)(std::asin(std::min(1.0, (double)k.S)) + 2e-5); }

lst_status build_geometry(const lst_params &p, const lst_module_desc *m, uint32_t n,
                          Geometry &g, std::string &err)
{
    if (!m || n == 0) { err = "empty module table"; return LST_ERR_INVALID_ARG; }
    if (!(p.B > 0) || !(p.pt_min > 0) || !(p.L >= 0) || !(p.sig_rphi >= 0) || !(p.sig_c >= 0) ||
        !(p.n_sigma >= 0)) {
        err = "parameters out of range";
        return LST_ERR_INVALID_ARG;
    }
    g = Geometry();
    g.n_mod = n;
    // ---- validation and surfaces ------------------------------------------
    uint32_t nb = 0, nd = 0;
    for (uint32_t i = 0; i < n; i++) {
        const lst_module_desc &d = m[i];
        if (!finite(d.s_lo) || !finite(d.s_hi) || !finite(d.c_min) || !finite(d.c_max) ||
            !finite(d.phi_min) || !finite(d.phi_max)) {
            err = "non-finite module field in module " + std::to_string(i);
            return LST_ERR_BAD_GEOMETRY;
        }
        if (!(d.phi_min >= 0 && d.phi_max <= kTwoPi + 1e-9 && d.phi_min < d.phi_max) ||
            !(d.c_min < d.c_max)) {
            err = "bad extent in module " + std::to_string(i);
            return LST_ERR_BAD_GEOMETRY;
        }
        if (d.kind == LST_BARREL) {
            if (d.side != 0 || !(d.s_lo > 0) || !(d.s_hi > d.s_lo)) {
                err = "bad barrel module " + std::to_string(i);
                return LST_ERR_BAD_GEOMETRY;
            }
            nb = std::max(nb, d.layer + 1);
        } else if (d.kind == LST_ENDCAP) {
            double zl = d.s_lo * d.side, zh = d.s_hi * d.side;
            if ((d.side != 1 && d.side != -1) || !(zl > p.L) || !(zh > zl) || !(d.c_min > 0)) {
                err = "bad endcap module " + std::to_string(i);
                return LST_ERR_BAD_GEOMETRY;
            }
            nd = std::max(nd, d.layer + 1);
        } else {
            err = "unknown module kind in module " + std::to_string(i);
            return LST_ERR_BAD_GEOMETRY;
        }
    }
    if (nb + 2 * nd > 64) { err = "too many surfaces"; return LST_ERR_BAD_GEOMETRY; }
    g.nb = nb;
    g.nd = nd;
    const uint32_t n_surf = nb + 2 * nd;
    // every module of a surface shares its sensor positions; surfaces move outward
    std::vector<double> surf_lo(n_surf, NAN), surf_hi(n_surf, NAN);
    g.kind.resize(n);
    g.surf.resize(n);
    for (uint32_t i = 0; i < n; i++) {
        const lst_module_desc &d = m[i];
        uint32_t s = d.kind == LST_BARREL ? d.layer : nb + (d.side > 0 ? 0 : nd) + d.layer;
        g.kind[i] = d.kind;
        g.surf[i] = s;
        if (std::isnan(surf_lo[s])) { surf_lo[s] = d.s_lo; surf_hi[s] = d.s_hi; }
        else if (surf_lo[s] != d.s_lo || surf_hi[s] != d.s_hi) {
            err = "modules of one surface disagree on sensor positions (module " + std::to_string(i) + ")";
            return LST_ERR_BAD_GEOMETRY;
        }
    }
    auto outward = [&](uint32_t s, uint32_t prev) {
        if (std::isnan(surf_lo[s]) || std::isnan(surf_lo[prev])) return true;
        return std::fabs(surf_lo[s]) > std::fabs(surf_hi[prev]);
    };
    bool ordered = true;
    for (uint32_t l = 1; l < nb; l++) ordered = ordered && outward(l, l - 1);
    for (uint32_t sd = 0; sd < 2; sd++)
        for (uint32_t d = 1; d < nd; d++) ordered = ordered && outward(nb + sd * nd + d, nb + sd * nd + d - 1);
    if (!ordered) {
        err = "surfaces are not ordered outward";
        return LST_ERR_BAD_GEOMETRY;
    }

    // ---- scalars -----------------------------------------------------------
    const double kmax = 0.299792458e-2 * p.B / p.pt_min;
    const double ns = p.n_sigma, rt2 = std::sqrt(2.0);
    double rmax = 0.0;
    for (uint32_t i = 0; i < n; i++)
        rmax = std::max(rmax, m[i].kind == LST_BARREL ? m[i].s_lo : m[i].c_max);
    Consts &c = g.c;
    c.L = (float)p.L;
    c.ec = (float)(p.n_sigma * p.sig_c);
    c.kmaxf = (float)kmax;
    c.khalf = (float)(kmax / 2.0);
    c.ns = (float)p.n_sigma;
    c.srp = (float)p.sig_rphi;
    c.sc = (float)p.sig_c;
    {
        // |f(x1) - f(x2)| <= |x1^2 - x2^2| f'(xm) / (2 xm): f(x) - 1 is a power
        // series in x^2 with non-negative coefficients; chords of a prompt
        // track never exceed the outermost anchor radius.
        double xm = rmax * kmax / 2.0;
        if (xm > 0.999) xm = 0.999;
        double fp = (xm / std::sqrt(1.0 - xm * xm) - std::asin(xm)) / (xm * xm);
        c.Kb = (float)(fp / (2.0 * xm) * kmax * kmax / 4.0);
    }
    c.B = p.B;
    c.n_sigma = p.n_sigma;
    c.sig_rphi = p.sig_rphi;
    c.sig_c = p.sig_c;
    c.kB = 0.299792458e-2 * p.B;
    c.n_mod = n;
    c.n_surf = n_surf;
    c.flags = p.flags;
    c.nphi = p.n_phi_bins ? p.n_phi_bins : 64;
    c.nkb = p.n_kappa_bins ? p.n_kappa_bins : 16;
    c.ls_group = p.ls_group ? p.ls_group : 6;
    c.ls_waves = p.ls_waves;
    c.kspan = (float)(1.25 * kmax);
    c.sk_cls[0] = 2e-4f;
    c.sk_cls[1] = 6e-4f;
    c.sk_cls[2] = 2e-3f;

    // ---- mini-doublet constants --------------------------------------------
    g.mdc.resize(n);
    for (uint32_t i = 0; i < n; i++) {
        const lst_module_desc &d = m[i];
        MdConst mc{0, 0, 0, 0};
        if (d.kind == LST_BARREL) {
            double r1 = d.s_lo, r2 = d.s_hi;
            double ph = half_turn(r2, kmax) - half_turn(r1, kmax) + ns * rt2 * p.sig_rphi / r1;
            mc.S = (float)std::sin(std::min(ph, kPi / 2));
            mc.G = (float)((r2 - r1) / std::cos(half_turn(r2, kmax)));
            mc.K = (float)(ns * rt2 * p.sig_c);
        } else {
            double z1 = std::fabs(d.s_lo), gap = std::fabs(d.s_hi) - std::fabs(d.s_lo);
            double rin = d.c_min, rout = d.c_max;
            // radial change between the sensors of an outgoing prompt track:
            // dr/dz = (dr/ds) s / (z - vz) <= r / (z - vz)
            double dr = gap * rout / (z1 - p.L);
            double ph = half_turn(rout + dr, kmax) - half_turn(rout, kmax) + ns * rt2 * p.sig_rphi / rin;
            mc.S = (float)std::sin(std::min(ph, kPi / 2));
            mc.D = (float)(dr + ns * rt2 * p.sig_c);
        }
        g.mdc[i] = mc;
    }

    // ---- module pairs: classes and the connection map ----------------------
    std::map<ZoneKey, uint32_t> zone_id;
    std::vector<uint32_t> zone(n);
    for (uint32_t i = 0; i < n; i++) {
        const lst_module_desc &d = m[i];
        ZoneKey k{d.kind, d.s_lo, d.s_hi, d.kind == LST_BARREL ? 0.0 : d.c_min,
                  d.kind == LST_BARREL ? 0.0 : d.c_max};
        auto it = zone_id.find(k);
        if (it == zone_id.end()) it = zone_id.emplace(k, (uint32_t)zone_id.size()).first;
        zone[i] = it->second;
    }
    const uint32_t nz = (uint32_t)zone_id.size();
    std::vector<int32_t> zpair_cls((size_t)nz * nz, -1);   // class id once a pair has an edge
    std::vector<LsClass> zpair_k((size_t)nz * nz);
    std::vector<uint8_t> zpair_done((size_t)nz * nz, 0);
    auto pair_class = [&](uint32_t A, uint32_t B) -> LsClass {
        const lst_module_desc &a = m[A], &b = m[B];
        bool bA = a.kind == LST_BARREL, bB = b.kind == LST_BARREL;
        double a_lo = bA ? a.s_lo : a.c_min;
        double b_hi = bB ? b.s_lo : b.c_max;
        LsClass k{};
        double ph = half_turn(b_hi, kmax) - half_turn(a_lo, kmax) + ns * rt2 * p.sig_rphi / a_lo;
        k.S = (float)std::sin(std::min(ph, kPi / 2));
        if (bA && bB) {
            double ra = a.s_lo, rb = b.s_lo, gA = a.s_hi - a.s_lo;
            k.type = 0;
            k.rho_lo = (float)(rb / ra);
            k.rho_hi = (float)(half_turn(rb, kmax) / half_turn(ra, kmax));
            double llo = (rb - ra) / gA;
            double lhi = std::sin(half_turn(rb, kmax) - half_turn(ra, kmax)) /
                         std::sin(half_turn(a.s_hi, kmax) - half_turn(ra, kmax));
            k.lam_lo = (float)llo;
            k.lam_hi = (float)lhi;
            k.tau = (float)(ns * rt2 * p.sig_rphi * (1.0 + std::max(llo, lhi)) / ra);
        } else if (!bA && !bB) {
            double zA = std::fabs(a.s_lo), zB = std::fabs(b.s_lo);
            double tlo = (zB + p.L) / (zA + p.L), thi = (zB - p.L) / (zA - p.L);
            double cf = 1.0 / arc_over_chord(b_hi * kmax / 2.0);
            k.type = 1;
            k.lo_fac = (float)(cf * tlo);
            k.hi_fac = (float)thi;
        } else {
            double zB = std::fabs(b.s_lo);
            k.type = 2;
            k.cf = (float)(1.0 / arc_over_chord(b_hi * kmax / 2.0));
            k.zs = b.s_lo > 0 ? 1.0f : -1.0f;
            k.zbpl = (float)(zB + p.L);
            k.zbml = (float)(zB - p.L);
        }
        return k;
    };

    std::vector<std::vector<uint32_t>> by_surf(n_surf);
    for (uint32_t i = 0; i < n; i++) by_surf[g.surf[i]].push_back(i);
    // surfaces a prompt outgoing track crosses right after s
    auto step = [&](uint32_t s) {
        std::vector<uint32_t> out;
        if (s < nb) {
            if (s + 1 < nb) out.push_back(s + 1);
            if (nd) { out.push_back(nb); out.push_back(nb + nd); }
        } else {
            uint32_t d = (s - nb) % nd;
            if (d + 1 < nd) out.push_back(s + 1);
        }
        return out;
    };
    // surfaces whose modules a segment from s may reach: one step, and with
    // skip-layer links also two (each surface once, in increasing order)
    const bool skip = (p.flags & LST_FLAG_SKIP_LAYER) != 0;
    auto next_surfaces = [&](uint32_t s) {
        std::vector<uint32_t> out = step(s);
        if (skip)
            for (uint32_t u : step(s))
                for (uint32_t t : step(u)) out.push_back(t);
        std::sort(out.begin(), out.end());
        out.erase(std::unique(out.begin(), out.end()), out.end());
        return out;
    };

    const double ec = p.n_sigma * p.sig_c;
    const double mz = kEdgeSigmas * p.sig_c;        // coarse-coordinate edge margin
    const double L = p.L;
    auto widen = [](double v) { return 1e-4 * (std::fabs(v) + 1.0); };

    g.edge_begin.assign(n + 1, 0);
    std::vector<std::vector<uint32_t>> edges(n);
    for (uint32_t A = 0; A < n; A++) {
        const lst_module_desc &a = m[A];
        bool bA = a.kind == LST_BARREL;
        double ra_min = bA ? a.s_lo : a.c_min;
        double mphiA = kEdgeSigmas * p.sig_rphi / ra_min + 1e-6;
        for (uint32_t t : next_surfaces(g.surf[A])) {
            for (uint32_t B : by_surf[t]) {
                const lst_module_desc &b = m[B];
                bool bB = b.kind == LST_BARREL;
                const size_t zp = (size_t)zone[A] * nz + zone[B];
                int32_t &cid = zpair_cls[zp];
                if (!zpair_done[zp]) { zpair_k[zp] = pair_class(A, B); zpair_done[zp] = 1; }
                const LsClass &k = zpair_k[zp];
                // azimuth: the anchors' azimuth difference is at most asin(S)
                double rb_min = bB ? b.s_lo : b.c_min;
                double mphiB = kEdgeSigmas * p.sig_rphi / rb_min + 1e-6;
                double phimax = std::asin(std::min(1.0, (double)k.S)) + 1e-5;
                if (arc_gap(a.phi_min - mphiA, a.phi_max + mphiA, b.phi_min - mphiB,
                            b.phi_max + mphiB) > phimax)
                    continue;
                bool ok;
                if (k.type == 0) {
                    double za0 = a.c_min - mz, za1 = a.c_max + mz;
                    double lo = INFINITY, hi = -INFINITY;
                    for (double rho : {(double)k.rho_lo, (double)k.rho_hi})
                        for (double v : {-L, L}) {
                            lo = std::min(lo, rho * (za0 - ec - v) + v);
                            hi = std::max(hi, rho * (za1 + ec - v) + v);
                        }
                    lo -= ec + widen(lo);
                    hi += ec + widen(hi);
                    ok = !(hi < b.c_min - mz || lo > b.c_max + mz);
                } else if (k.type == 1) {
                    double ra0 = a.c_min - mz, ra1 = a.c_max + mz;
                    double lo = k.lo_fac * (ra0 - ec) - ec, hi = k.hi_fac * (ra1 + ec) + ec;
                    lo -= widen(lo);
                    hi += widen(hi);
                    ok = !(hi < b.c_min - mz || lo > b.c_max + mz);
                } else {
                    double za0 = a.c_min - mz, za1 = a.c_max + mz;
                    double zap0 = k.zs > 0 ? za0 : -za1, zap1 = k.zs > 0 ? za1 : -za0;
                    double ra0 = a.s_lo - 0.01, ra1 = a.s_lo + 0.01;
                    if (!(zap1 + ec + L > 0)) {
                        ok = false;
                    } else {
                        double lo = k.cf * (k.zbpl / (zap1 + ec + L)) * ra0 - ec;
                        double hi = INFINITY;
                        if (zap0 - ec - L > 0) hi = (k.zbml / (zap0 - ec - L)) * ra1 + ec;
                        lo -= widen(lo);
                        hi += widen(hi);
                        ok = !(hi < b.c_min - mz || lo > b.c_max + mz);
                    }
                }
                if (!ok) continue;
                if (cid < 0) {
                    cid = (int32_t)g.classes.size();
                    g.classes.push_back(k);
                }
                edges[A].push_back(B);
                edges[A].push_back((uint32_t)cid);
            }
        }
    }
    for (uint32_t A = 0; A < n; A++) g.edge_begin[A + 1] = g.edge_begin[A] + (uint32_t)edges[A].size() / 2;
    g.edge_dst.resize(g.edge_begin[n]);
    g.edge_cls.resize(g.edge_begin[n]);
    for (uint32_t A = 0; A < n; A++) {
        // destinations in increasing module order, so that segments come out
        // sorted by their outer mini-doublet
        std::vector<std::pair<uint32_t, uint32_t>> e;
        for (size_t i = 0; i < edges[A].size(); i += 2) e.emplace_back(edges[A][i], edges[A][i + 1]);
        std::sort(e.begin(), e.end());
        for (size_t i = 0; i < e.size(); i++) {
            g.edge_dst[g.edge_begin[A] + i] = e[i].first;
            g.edge_cls[g.edge_begin[A] + i] = e[i].second;
        }
    }

    // azimuth extent of every module with the margin the map uses for an
    // outer module: a segment's outer anchor lies within it
    g.mod_phi.resize(2 * (size_t)n);
    for (uint32_t B = 0; B < n; B++) {
        const lst_module_desc &b = m[B];
        const double rb_min = b.kind == LST_BARREL ? b.s_lo : b.c_min;
        const double mphiB = kEdgeSigmas * p.sig_rphi / rb_min + 1e-6;
        double c = 0.5 * (b.phi_min + b.phi_max);
        if (c > kPi) c -= kTwoPi;
        g.mod_phi[2 * (size_t)B] = (float)c;
        g.mod_phi[2 * (size_t)B + 1] = (float)(0.5 * (b.phi_max - b.phi_min) + mphiB);
    }

    // segment-walk runs.  Module k of a run (destination first + k) has its
    // azimuth centre within dev of phi0 + k * pitch (binary32 values as
    // stored, the difference taken in binary64); the window is the largest
    // half-width plus the class's reach plus dev plus 1e-4 for the binary32
    // arithmetic of the run test (stored in module indices, i.e. divided by
    // the pitch, for runs of more than one module), so every module the
    // per-module reach test accepts lies in the run's accepted index range.  Runs end where the
    // destinations stop being consecutive, the class changes, a centre
    // strays by more than 1e-3 from the pitch, or the span plus the window
    // nears half a turn (the run test takes no wrap-around past the span).
    g.run_begin.assign(n + 1, 0);
    g.run_rec.clear();
    g.run_win.clear();
    for (uint32_t A = 0; A < n; A++) {
        const uint32_t e0 = g.edge_begin[A], e1 = g.edge_begin[A + 1];
        for (uint32_t i = e0; i < e1;) {
            const uint32_t first = g.edge_dst[i], cid = g.edge_cls[i];
            const float reach = ls_reach(g.classes[cid]);
            const double c0 = g.mod_phi[2 * (size_t)first];
            double hw = g.mod_phi[2 * (size_t)first + 1];
            double pitch = 0.0, u = 0.0;   // unwrapped centre of the last module, relative to c0
            uint32_t len = 1;
            while (i + len < e1 && len < 255u && g.edge_dst[i + len] == first + len && g.edge_cls[i + len] == cid) {
                const uint32_t B = first + len;
                const double step = wrap_pi(g.mod_phi[2 * (size_t)B] - g.mod_phi[2 * (size_t)B - 2]);
                if (len == 1) {
                    if (std::fabs(step) < 1e-4 || std::fabs(step) > 0.5) break;
                    pitch = step;
                } else if (std::fabs(u + step - len * pitch) > 1e-3) {
                    break;
                }
                const double hwb = std::max(hw, (double)g.mod_phi[2 * (size_t)B + 1]);
                if (std::fabs(u + step) + hwb + reach + 2e-3 > 3.0) break;
                u += step;
                hw = hwb;
                len++;
            }
            if (len > 1) pitch = u / (len - 1);
            // the run test uses the inverse pitch as stored: the pitch it
            // implies is 1 / invf, and the deviations are taken from it
            const float phi0f = (float)c0, invf = len > 1 ? (float)(1.0 / pitch) : 0.0f;
            const double pitch_used = len > 1 ? 1.0 / (double)invf : 0.0;
            double dev = 0.0;
            for (uint32_t k = 1; k < len; k++)
                dev = std::max(dev, std::fabs(wrap_pi(g.mod_phi[2 * (size_t)(first + k)] -
                                                      ((double)phi0f + k * pitch_used))));
            uint32_t rec[4] = {first, cid | (len << 24), 0u, 0u};
            std::memcpy(&rec[2], &phi0f, 4);
            std::memcpy(&rec[3], &invf, 4);
            g.run_rec.insert(g.run_rec.end(), rec, rec + 4);
            // window in radians for a single module, else in module indices
            const double win = hw + reach + dev + 1e-4;
            g.run_win.push_back((float)(len > 1 ? win * std::fabs((double)invf) : win));
            i += len;
        }
        g.run_begin[A + 1] = (uint32_t)g.run_win.size();
    }

    // extent of every module as the ingest check reads it: azimuth centre in
    // (-pi, pi] and half-width, coarse-coordinate range, each widened by
    // kHitSigmas resolutions; the two sensor positions and their tolerance
    g.mod_ext.resize(8 * (size_t)n);
    for (uint32_t i = 0; i < n; i++) {
        const lst_module_desc &d = m[i];
        const double r_min = d.kind == LST_BARREL ? d.s_lo : d.c_min;
        double c = 0.5 * (d.phi_min + d.phi_max);
        if (c > kPi) c -= kTwoPi;
        float *e = &g.mod_ext[8 * (size_t)i];
        e[0] = (float)c;
        e[1] = (float)(0.5 * (d.phi_max - d.phi_min) + kHitSigmas * p.sig_rphi / r_min);
        e[2] = (float)(d.c_min - kHitSigmas * p.sig_c);
        e[3] = (float)(d.c_max + kHitSigmas * p.sig_c);
        e[4] = (float)d.s_lo;
        e[5] = (float)d.s_hi;
        e[6] = (float)kSurfTol;
        e[7] = d.kind == LST_BARREL ? 0.0f : 1.0f;
    }

    // ---- surfaces for the seed lookup --------------------------------------
    g.surfaces.assign(n_surf, Surface{});
    std::vector<bool> seen(n_surf, false);
    for (uint32_t i = 0; i < n; i++) {
        const lst_module_desc &d = m[i];
        Surface &s = g.surfaces[g.surf[i]];
        float r1, r2, z1, z2;
        if (d.kind == LST_BARREL) {
            r1 = (float)(d.s_lo - 0.05);
            r2 = (float)(d.s_lo + 0.05);
            z1 = (float)(d.c_min - mz - 0.5);
            z2 = (float)(d.c_max + mz + 0.5);
        } else {
            r1 = (float)(d.c_min - mz - 0.5);
            r2 = (float)(d.c_max + mz + 0.5);
            z1 = z2 = (float)d.s_lo;
        }
        if (!seen[g.surf[i]]) {
            s.kind = d.kind; s.side = d.side; s.r1 = r1; s.r2 = r2; s.z1 = z1; s.z2 = z2;
            seen[g.surf[i]] = true;
        } else {
            s.r1 = std::min(s.r1, r1); s.r2 = std::max(s.r2, r2);
            s.z1 = std::min(s.z1, z1); s.z2 = std::max(s.z2, z2);
        }
    }
    for (uint32_t s = 0; s < n_surf; s++)
        if (!seen[s]) { g.surfaces[s].kind = 2; }   // empty surface
    return LST_OK;
}

// ---- geometry cache ---------------------------------------------------------
//
// Blob: magic, the key (the parameters with the stream pointer cleared, then
// the module table, byte for byte), then every table of the Geometry.  The
// file name carries a 64-bit FNV-1a hash of the key; a blob is used only when
// its key equals the inputs' exactly and it parses to its last byte.

namespace {

constexpr char kBlobMagic[8] = {'L', 'S', 'T', 'G', 'E', 'O', '0', '1'};

uint64_t fnv1a64(const std::string &s)
{
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

struct BlobWriter {
    std::string out;
    template <typename T>
    void pod(const T &v) { out.append(reinterpret_cast<const char *>(&v), sizeof(T)); }
    template <typename T>
    void vec(const std::vector<T> &v)
    {
        pod<uint64_t>(v.size());
        if (!v.empty()) out.append(reinterpret_cast<const char *>(v.data()), v.size() * sizeof(T));
    }
};

struct BlobReader {
    const char *p, *end;
    bool ok = true;
    template <typename T>
    void pod(T &v)
    {
        if (!ok || (size_t)(end - p) < sizeof(T)) { ok = false; return; }
        std::memcpy(&v, p, sizeof(T));
        p += sizeof(T);
    }
    template <typename T>
    void vec(std::vector<T> &v)
    {
        uint64_t n = 0;
        pod(n);
        if (!ok || n > (uint64_t)(end - p) / sizeof(T)) { ok = false; return; }
        v.resize(n);
        if (n) std::memcpy(v.data(), p, n * sizeof(T));
        p += n * sizeof(T);
    }
};

// every table of the Geometry, in one order for writing and reading
template <typename IO>
void geometry_fields(IO &io, Geometry &g)
{
    io.pod(g.n_mod);
    io.pod(g.nb);
    io.pod(g.nd);
    io.vec(g.kind);
    io.vec(g.surf);
    io.vec(g.mdc);
    io.vec(g.edge_begin);
    io.vec(g.edge_dst);
    io.vec(g.edge_cls);
    io.vec(g.classes);
    io.vec(g.run_begin);
    io.vec(g.run_rec);
    io.vec(g.run_win);
    io.vec(g.mod_phi);
    io.vec(g.mod_ext);
    io.vec(g.surfaces);
    io.pod(g.c);
}

std::string geometry_key(const lst_params &p, const lst_module_desc *m, uint32_t n)
{
    lst_params q;
    std::memcpy(&q, &p, sizeof q);
    q.stream = nullptr;
    std::string key(reinterpret_cast<const char *>(&q), sizeof q);
    key.append(reinterpret_cast<const char *>(m), (size_t)n * sizeof(lst_module_desc));
    return key;
}

bool read_file(const std::string &path, std::string &data)
{
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    bool ok = std::fseek(f, 0, SEEK_END) == 0;
    const long sz = ok ? std::ftell(f) : -1;
    ok = ok && sz >= 0 && std::fseek(f, 0, SEEK_SET) == 0;
    if (ok) {
        data.resize((size_t)sz);
        ok = std::fread(&data[0], 1, data.size(), f) == data.size();
    }
    std::fclose(f);
    return ok;
}

}  // namespace

lst_status build_geometry_cached(const lst_params &p, const lst_module_desc *m, uint32_t n,
                                 const std::string &dir, Geometry &g, std::string &err, bool &from_cache)
{
    from_cache = false;
    if (dir.empty() || !m || n == 0) return build_geometry(p, m, n, g, err);
    const std::string key = geometry_key(p, m, n);
    char name[64];
    std::snprintf(name, sizeof name, "/lst_geometry_%016llx.bin", (unsigned long long)fnv1a64(key));
    const std::string path = dir + name;
    std::string data;
    if (read_file(path, data) && data.size() >= sizeof kBlobMagic + 8 &&
        std::memcmp(data.data(), kBlobMagic, sizeof kBlobMagic) == 0) {
        BlobReader r{data.data() + sizeof kBlobMagic, data.data() + data.size()};
        uint64_t klen = 0;
        r.pod(klen);
        if (r.ok && klen == key.size() && (uint64_t)(r.end - r.p) >= klen && std::memcmp(r.p, key.data(), klen) == 0) {
            r.p += klen;
            Geometry h;
            geometry_fields(r, h);
            if (r.ok && r.p == r.end && h.n_mod == n) {
                g = std::move(h);
                from_cache = true;
                return LST_OK;
            }
        }
    }
    const lst_status st = build_geometry(p, m, n, g, err);
    if (st != LST_OK) return st;
    BlobWriter w;
    w.out.append(kBlobMagic, sizeof kBlobMagic);
    w.pod<uint64_t>(key.size());
    w.out += key;
    geometry_fields(w, g);
    // written beside, then renamed over the blob: readers never see a part
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid()) + "_" +
                            std::to_string((unsigned long long)(uintptr_t)&w);
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (f) {
        const bool ok = std::fwrite(w.out.data(), 1, w.out.size(), f) == w.out.size();
        if (std::fclose(f) == 0 && ok) {
            if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
        } else {
            std::remove(tmp.c_str());
        }
    }
    return LST_OK;
}

}  // namespace lst
