// Host-side check of the geometry builder, built with the address and
// undefined-behaviour sanitizers by tests/test_sanitizers.py: reads a module
// table and parameters (raw lst_module_desc / lst_params records), builds the
// geometry, connection map and segment-walk runs, and checks that the runs
// cover every edge in order.  Exit status 0 when everything holds.
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

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
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
    std::printf("modules %u edges %zu runs %zu classes %zu\n", g.n_mod, g.edge_dst.size(), g.run_win.size(),
                g.classes.size());
    return 0;
}
