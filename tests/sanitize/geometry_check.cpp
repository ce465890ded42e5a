// Host-side check of the geometry builder, built with the address and
// undefined-behaviour sanitizers by tests/test_sanitizers.py: reads a module
// table and parameters (raw lst_module_desc / lst_params records), builds the
// geometry, connection map and segment-walk runs, and checks that the runs
// cover every edge in order; with a third argument (a directory), that the
// geometry cache writes a blob on a miss, reads the same tables back on a
// hit and misses for other parameters.  Exit status 0 when everything holds.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lst_internal.h"

static bool read_file(const char *path, std::vector<char> &buf)
{
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long n = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    buf.resize(n > 0 ? (size_t)n : 0);
    const bool ok = n >= 0 && std::fread(buf.data(), 1, buf.size(), f) == buf.size();
    std::fclose(f);
    return ok;
}

template <typename T>
static bool same_vec(const std::vector<T> &a, const std::vector<T> &b)
{
    return a.size() == b.size() && (a.empty() || std::memcmp(a.data(), b.data(), a.size() * sizeof(T)) == 0);
}

static bool same_geometry(const lst::Geometry &a, const lst::Geometry &b)
{
    return a.n_mod == b.n_mod && a.nb == b.nb && a.nd == b.nd && same_vec(a.kind, b.kind) &&
           same_vec(a.surf, b.surf) && same_vec(a.mdc, b.mdc) && same_vec(a.edge_begin, b.edge_begin) &&
           same_vec(a.edge_dst, b.edge_dst) && same_vec(a.edge_cls, b.edge_cls) && same_vec(a.classes, b.classes) &&
           same_vec(a.run_begin, b.run_begin) && same_vec(a.run_rec, b.run_rec) && same_vec(a.run_win, b.run_win) &&
           same_vec(a.mod_phi, b.mod_phi) && same_vec(a.mod_ext, b.mod_ext) && same_vec(a.surfaces, b.surfaces) &&
           std::memcmp(&a.c, &b.c, sizeof a.c) == 0;
}

int main(int argc, char **argv)
{
    if (argc != 3 && argc != 4) return 2;
    std::vector<char> mods, prm;
    if (!read_file(argv[1], mods) || !read_file(argv[2], prm) || prm.size() != sizeof(lst_params) ||
        mods.size() % sizeof(lst_module_desc))
        return 2;
    lst_params p;
    std::memcpy(&p, prm.data(), sizeof p);
    const uint32_t n = (uint32_t)(mods.size() / sizeof(lst_module_desc));
    std::vector<lst_module_desc> m(n);
    std::memcpy(m.data(), mods.data(), mods.size());
    lst::Geometry g;
    std::string err;
    const lst_status st = lst::build_geometry(p, m.data(), n, g, err);
    if (st != LST_OK) {
        std::printf("build_geometry: %d %s\n", (int)st, err.c_str());
        return 1;
    }
    // the runs of every module cover its edges in order: run r holds the
    // edges to first, first + 1, ... of one class
    size_t e = 0;
    for (uint32_t a = 0; a < g.n_mod; a++) {
        if (e != g.edge_begin[a]) return 3;
        for (uint32_t r = g.run_begin[a]; r < g.run_begin[a + 1]; r++) {
            const uint32_t first = g.run_rec[4 * (size_t)r], cls = g.run_rec[4 * (size_t)r + 1] & 0xFFFFFFu;
            const uint32_t len = g.run_rec[4 * (size_t)r + 1] >> 24;
            if (len == 0) return 4;
            for (uint32_t k = 0; k < len; k++, e++)
                if (e >= g.edge_begin[a + 1] || g.edge_dst[e] != first + k || g.edge_cls[e] != cls) return 5;
        }
        if (e != g.edge_begin[a + 1]) return 6;
    }
    // with a cache directory: the first cached build writes a blob, the
    // second reads it back, and both equal the tables built without a cache
    if (argc == 4) {
        lst::Geometry g1, g2;
        bool hit1 = true, hit2 = false;
        if (lst::build_geometry_cached(p, m.data(), n, argv[3], g1, err, hit1) != LST_OK || hit1) return 7;
        if (lst::build_geometry_cached(p, m.data(), n, argv[3], g2, err, hit2) != LST_OK || !hit2) return 8;
        if (!same_geometry(g, g1) || !same_geometry(g, g2)) return 9;
        // other parameters: a miss, not the blob of the first
        lst_params q = p;
        q.n_sigma += 0.5;
        lst::Geometry g3;
        bool hit3 = true;
        if (lst::build_geometry_cached(q, m.data(), n, argv[3], g3, err, hit3) != LST_OK || hit3) return 10;
        std::printf("cache: miss, hit, miss for other parameters\n");
    }
    std::printf("modules %u edges %zu runs %zu classes %zu\n", g.n_mod, g.edge_dst.size(), g.run_win.size(),
                g.classes.size());
    return 0;
}
