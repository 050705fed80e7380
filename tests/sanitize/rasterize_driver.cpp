// Host driver for the sanitizer check of the rasterizer (test infrastructure).
//
// Built with g++ -fsanitize=address,undefined together with the library's
// csrc/geometry.cpp, it reads one geometry from stdin and writes what
// lq::rasterize produced to stdout, so that a test can run every host
// geometry case through an instrumented build and compare the result with
// the library's own lq_rasterize.
//
// stdin:  lq_params, int32 n_objs, lq_object[n_objs], int64 n_recs,
//         lq_site_anchor[n_recs], int64 n_object_sites, int64[n_object_sites]
// stdout: int32 rc; when rc == 0: int64 N, int64 n_sim, uint8 type[N],
//         uint8 mask[N], int64 n_anch, int64 site[n_anch],
//         double data[n_anch * ANCH_STRIDE]
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "lq_internal.h"

template <typename T>
static bool get(T* p, size_t n) {
    return n == 0 || std::fread(p, sizeof(T), n, stdin) == n;
}
template <typename T>
static void put(const T* p, size_t n) {
    if (n) std::fwrite(p, sizeof(T), n, stdout);
}

int main() {
    lq_params p{};
    int32_t n_objs = 0;
    int64_t n_recs = 0, n_os = 0;
    if (!get(&p, 1) || !get(&n_objs, 1) || n_objs < 0) return 2;
    std::vector<lq_object> objs((size_t)n_objs);
    if (!get(objs.data(), objs.size()) || !get(&n_recs, 1) || n_recs < 0) return 2;
    std::vector<lq_site_anchor> recs((size_t)n_recs);
    if (!get(recs.data(), recs.size()) || !get(&n_os, 1) || n_os < 0) return 2;
    std::vector<int64_t> os((size_t)n_os);
    if (!get(os.data(), os.size())) return 2;
    // S0 of Eq. (S0def): the nematic root of 2A + B S + 3 C S^2 = 0
    const double disc = p.B * p.B - 24.0 * p.A * p.C;
    const double S0 = (p.C > 0.0 && disc >= 0.0) ? (-p.B + std::sqrt(disc)) / (6.0 * p.C) : NAN;
    lq::Geometry g;
    std::string err;
    const int32_t rc = lq::rasterize(p, S0, objs.data(), n_objs, recs.data(), n_recs, os.data(), n_os, g, err);
    put(&rc, 1);
    if (rc != LQ_OK) {
        std::fprintf(stderr, "%s\n", err.c_str());
        return 0;
    }
    const int64_t N = (int64_t)g.type.size(), n_anch = (int64_t)g.anch_site.size();
    put(&N, 1);
    put(&g.n_sim, 1);
    put(g.type.data(), g.type.size());
    put(g.mask.data(), g.mask.size());
    put(&n_anch, 1);
    put(g.anch_site.data(), g.anch_site.size());
    put(g.anch_data.data(), g.anch_data.size());
    return 0;
}
