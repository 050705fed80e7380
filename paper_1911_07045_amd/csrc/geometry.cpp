// Host rasterizer of liblqfire: objects and per-site records -> site types,
// neighbour masks and per-site anchoring forms.
//
// Site typing follows sec. III.B (bulk, boundary, inside an object; only
// bulk and boundary sites are simulated).  Anchoring follows sec. II.A.4:
//   - Nobili-Durand W tr((Q - Q0)^2), Q0 = 3/2 S0 (n0 n0 - I/3); a
//     Rapini-Papoular strength W >= 0 enters as W / (9 S0^2);
//   - Fournier-Galatola W |Qt - P Qt P|^2, Qt = Q + S0/2 I, P = I - nu nu
//     (degenerate planar); a Rapini-Papoular strength W < 0 enters as
//     |W| / (9 S0^2).
// Both are quadratic in the five components q, so the terms of one site are
// summed into one form f = 1/2 q^T K q + b^T q + c, stored as the upper
// triangle of K (15 values), b (5) and c (1); the kernels take the force
// -(K q + b) and the energy from it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lq_internal.h"

namespace lq {
namespace {

struct Lat {
    int64_t n[3];
    bool per[3];
    int64_t N() const { return n[0] * n[1] * n[2]; }
    int64_t idx(int64_t x, int64_t y, int64_t z) const { return x + n[0] * (y + n[1] * z); }
    // neighbour of (c) one step along axis k in direction s, -1 off an open edge
    int64_t nbr(const int64_t c[3], int k, int s) const {
        int64_t e[3] = {c[0], c[1], c[2]};
        e[k] += s;
        if (e[k] < 0 || e[k] >= n[k]) {
            if (!per[k]) return -1;
            e[k] = (e[k] + n[k]) % n[k];
        }
        return idx(e[0], e[1], e[2]);
    }
};

double min_image(double d, int64_t n, bool periodic) {
    if (!periodic) return d;
    double nn = (double)n;
    return d - nn * std::floor(d / nn + 0.5);
}

// q components of 3/2 S (n n - I/3)
void q_of(const double nv[3], double S, double out[5]) {
    double h = 1.5 * S;
    out[0] = h * (nv[0] * nv[0] - 1.0 / 3.0);
    out[1] = h * nv[0] * nv[1];
    out[2] = h * nv[0] * nv[2];
    out[3] = h * (nv[1] * nv[1] - 1.0 / 3.0);
    out[4] = h * nv[1] * nv[2];
}

// The symmetric traceless tensor of the unit q component a (Qzz = -Qxx - Qyy).
void basis(int a, double E[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) E[i][j] = 0.0;
    switch (a) {
        case 0: E[0][0] = 1.0; E[2][2] = -1.0; break;
        case 1: E[0][1] = E[1][0] = 1.0; break;
        case 2: E[0][2] = E[2][0] = 1.0; break;
        case 3: E[1][1] = 1.0; E[2][2] = -1.0; break;
        default: E[1][2] = E[2][1] = 1.0; break;
    }
}

double frob(const double X[3][3], const double Y[3][3]) {
    double s = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s += X[i][j] * Y[i][j];
    return s;
}

// position of K[a][b] (a <= b) in the stored upper triangle
int tri(int a, int b) { return a * 5 - a * (a - 1) / 2 + (b - a); }

// d += form of W tr((Q - Q0)^2) = W (q - q0)^T M (q - q0), M_ab = E_a : E_b
void add_nd(double* d, double W, const double q0[5]) {
    double E[5][3][3];
    for (int a = 0; a < 5; ++a) basis(a, E[a]);
    double M[5][5];
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) M[a][b] = frob(E[a], E[b]);
    for (int a = 0; a < 5; ++a) {
        for (int b = a; b < 5; ++b) d[tri(a, b)] += 2.0 * W * M[a][b];
        double Mq0 = 0.0;
        for (int b = 0; b < 5; ++b) Mq0 += M[a][b] * q0[b];
        d[15 + a] += -2.0 * W * Mq0;
        d[20] += W * q0[a] * Mq0;
    }
}

// d += form of W |D|^2, D = L(q) + D0, L_a = E_a - P E_a P, D0 = S0/2 nu nu
void add_fg(double* d, double W, const double nu[3], double S0) {
    double P[3][3], D0[3][3], Lb[5][3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            P[i][j] = (i == j ? 1.0 : 0.0) - nu[i] * nu[j];
            D0[i][j] = 0.5 * S0 * nu[i] * nu[j];
        }
    for (int a = 0; a < 5; ++a) {
        double E[3][3];
        basis(a, E);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) s += P[i][k] * E[k][l] * P[l][j];
                Lb[a][i][j] = E[i][j] - s;
            }
    }
    for (int a = 0; a < 5; ++a) {
        for (int b = a; b < 5; ++b) d[tri(a, b)] += 2.0 * W * frob(Lb[a], Lb[b]);
        d[15 + a] += 2.0 * W * frob(Lb[a], D0);
    }
    d[20] += W * frob(D0, D0);
}

bool normalize(const double in[3], double out[3]) {
    double r = std::sqrt(in[0] * in[0] + in[1] * in[1] + in[2] * in[2]);
    if (!(r > 0.0) || !std::isfinite(r)) return false;
    out[0] = in[0] / r;
    out[1] = in[1] / r;
    out[2] = in[2] / r;
    return true;
}

// kind of term (false: Nobili-Durand, true: Fournier-Galatola) and its strength
bool strength(int32_t law, double W, double S0, bool* fg, double* out, std::string& err) {
    if (!std::isfinite(W)) {
        err = "anchoring strength is not finite";
        return false;
    }
    *fg = false;
    if (law == LQ_LAW_ND) {
        *out = W;
    } else if (law == LQ_LAW_RP) {
        *fg = W < 0.0;
        *out = std::fabs(W) / (9.0 * S0 * S0);
    } else if (law == LQ_LAW_FG) {
        *fg = true;
        *out = W;
    } else {
        err = "unknown anchoring law";
        return false;
    }
    if (*out < 0.0) {
        err = "negative Nobili-Durand or Fournier-Galatola strength";
        return false;
    }
    return true;
}

bool inside(const lq_object& o, const Lat& L, int64_t x, int64_t y, int64_t z) {
    if (o.kind == LQ_OBJ_WALL || o.kind == LQ_OBJ_PATTERNED_WALL) {
        int64_t c[3] = {x, y, z};
        return c[o.axis] == o.plane;
    }
    double dx = min_image((double)x - o.center[0], L.n[0], L.per[0]);
    double dy = min_image((double)y - o.center[1], L.n[1], L.per[1]);
    double dz = min_image((double)z - o.center[2], L.n[2], L.per[2]);
    return dx * dx + dy * dy + dz * dz < o.radius * o.radius;
}

// Sites inside a sphere: scan the bounding box (wrapping on periodic axes).
void sphere_sites(const lq_object& o, const Lat& L, std::vector<int64_t>& out) {
    int64_t lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = (int64_t)std::floor(o.center[k] - o.radius) - 1;
        hi[k] = (int64_t)std::ceil(o.center[k] + o.radius) + 1;
        if (!L.per[k]) {
            lo[k] = std::max<int64_t>(lo[k], 0);
            hi[k] = std::min<int64_t>(hi[k], L.n[k] - 1);
        } else if (hi[k] - lo[k] + 1 >= L.n[k]) {
            lo[k] = 0;
            hi[k] = L.n[k] - 1;
        }
    }
    for (int64_t z = lo[2]; z <= hi[2]; ++z)
        for (int64_t y = lo[1]; y <= hi[1]; ++y)
            for (int64_t x = lo[0]; x <= hi[0]; ++x) {
                int64_t w[3] = {x, y, z};
                for (int k = 0; k < 3; ++k) w[k] = ((w[k] % L.n[k]) + L.n[k]) % L.n[k];
                if (inside(o, L, w[0], w[1], w[2])) out.push_back(L.idx(w[0], w[1], w[2]));
            }
}

void object_interior(const lq_object& o, const Lat& L, std::vector<int64_t>& out) {
    out.clear();
    if (o.kind == LQ_OBJ_SPHERE) {
        sphere_sites(o, L, out);
        return;
    }
    int a = o.axis, b = (a + 1) % 3, c = (a + 2) % 3;
    for (int64_t j = 0; j < L.n[c]; ++j)
        for (int64_t i = 0; i < L.n[b]; ++i) {
            int64_t w[3];
            w[a] = o.plane;
            w[b] = i;
            w[c] = j;
            out.push_back(L.idx(w[0], w[1], w[2]));
        }
}

// surface normal of object o seen from boundary site (x, y, z)
void surface_normal(const lq_object& o, const Lat& L, int64_t x, int64_t y, int64_t z, double nu[3]) {
    nu[0] = nu[1] = nu[2] = 0.0;
    if (o.kind == LQ_OBJ_WALL || o.kind == LQ_OBJ_PATTERNED_WALL) {
        nu[o.axis] = 1.0;
        return;
    }
    double d[3] = {min_image((double)x - o.center[0], L.n[0], L.per[0]),
                   min_image((double)y - o.center[1], L.n[1], L.per[1]),
                   min_image((double)z - o.center[2], L.n[2], L.per[2])};
    double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    nu[0] = d[0] / r;
    nu[1] = d[1] / r;
    nu[2] = d[2] / r;
}

// preferred director of object o at boundary site (x, y, z)
void preferred_director(const lq_object& o, const Lat& L, int64_t x, int64_t y, int64_t z,
                        double n0[3]) {
    if (o.kind == LQ_OBJ_PATTERNED_WALL) {
        int a = o.axis;
        int u = a == 0 ? 1 : 0;
        int w = a == 2 ? 1 : 2;
        int64_t c[3] = {x, y, z};
        double best = INFINITY, bu = 0.0, bw = 0.0;
        for (int i = 0; i < o.count[0]; ++i)
            for (int j = 0; j < o.count[1]; ++j) {
                double du = min_image((double)c[u] - (o.offset[0] + o.pitch[0] * i), L.n[u], L.per[u]);
                double dw = min_image((double)c[w] - (o.offset[1] + o.pitch[1] * j), L.n[w], L.per[w]);
                double d2 = du * du + dw * dw;
                if (d2 < best) {
                    best = d2;
                    bu = du;
                    bw = dw;
                }
            }
        double r = std::sqrt(bu * bu + bw * bw);
        n0[0] = n0[1] = n0[2] = 0.0;
        n0[u] = bu / r;
        n0[w] = bw / r;
        return;
    }
    double nu[3];
    surface_normal(o, L, x, y, z, nu);
    if (o.dir_mode == LQ_DIR_FIXED) {
        normalize(o.dir, n0);
    } else {
        n0[0] = nu[0];
        n0[1] = nu[1];
        n0[2] = nu[2];
    }
}

bool check_object(const lq_object& o, const Lat& L, std::string& err) {
    if (o.kind == LQ_OBJ_WALL || o.kind == LQ_OBJ_PATTERNED_WALL) {
        if (o.axis < 0 || o.axis > 2) {
            err = "wall axis out of range";
            return false;
        }
        if (o.plane < 0 || o.plane >= L.n[o.axis]) {
            err = "wall plane out of range";
            return false;
        }
        if (o.kind == LQ_OBJ_PATTERNED_WALL) {
            if (o.count[0] < 1 || o.count[1] < 1 || !std::isfinite(o.pitch[0]) ||
                !std::isfinite(o.pitch[1]) || !std::isfinite(o.offset[0]) ||
                !std::isfinite(o.offset[1])) {
                err = "bad patterned-wall array";
                return false;
            }
        }
    } else if (o.kind == LQ_OBJ_SPHERE) {
        if (!(o.radius > 0.0) || !std::isfinite(o.radius) || !std::isfinite(o.center[0]) ||
            !std::isfinite(o.center[1]) || !std::isfinite(o.center[2])) {
            err = "bad sphere";
            return false;
        }
    } else {
        err = "unknown object kind";
        return false;
    }
    if (o.kind != LQ_OBJ_PATTERNED_WALL) {
        if (o.dir_mode == LQ_DIR_FIXED) {
            double t[3];
            if (!normalize(o.dir, t)) {
                err = "fixed anchoring direction is zero or not finite";
                return false;
            }
        } else if (o.dir_mode != LQ_DIR_NORMAL) {
            err = "unknown director mode";
            return false;
        }
    }
    return true;
}

}  // namespace

int rasterize(const lq_params& p, double S0, const lq_object* objs, int32_t n_objs,
              const lq_site_anchor* recs, int64_t n_recs, const int64_t* object_sites,
              int64_t n_object_sites, Geometry& g, std::string& err) {
    Lat L;
    for (int k = 0; k < 3; ++k) {
        L.n[k] = p.n[k];
        L.per[k] = p.periodic[k] != 0;
    }
    const int64_t N = L.N();
    if (n_objs < 0 || n_recs < 0 || n_object_sites < 0 || (n_objs > 0 && !objs) ||
        (n_recs > 0 && !recs) || (n_object_sites > 0 && !object_sites)) {
        err = "bad geometry array arguments";
        return LQ_EINVAL;
    }
    bool anchoring = n_recs > 0;
    for (int32_t i = 0; i < n_objs; ++i) {
        if (!check_object(objs[i], L, err)) return LQ_EINVAL;
        anchoring = true;
    }
    if (anchoring && !(std::isfinite(S0) && S0 > 0.0)) {
        err = "anchoring needs a positive real S0 (check A, B, C)";
        return LQ_EINVAL;
    }
    g.type.assign((size_t)N, 0);
    std::vector<std::vector<int64_t>> interior((size_t)n_objs);
    for (int32_t i = 0; i < n_objs; ++i) {
        object_interior(objs[i], L, interior[i]);
        for (int64_t s : interior[i]) g.type[s] = 2;
    }
    for (int64_t i = 0; i < n_object_sites; ++i) {
        int64_t s = object_sites[i];
        if (s < 0 || s >= N) {
            err = "object site out of range";
            return LQ_EINVAL;
        }
        g.type[s] = 2;
    }
    // per-site anchoring forms, indexed by site through a sparse map
    std::vector<int64_t> slot((size_t)N, -1);
    std::vector<int64_t> sites;
    std::vector<double> data;
    auto row = [&](int64_t s) -> double* {
        if (slot[s] < 0) {
            slot[s] = (int64_t)sites.size();
            sites.push_back(s);
            data.insert(data.end(), ANCH_STRIDE, 0.0);
        }
        return &data[ANCH_STRIDE * slot[s]];
    };
    std::vector<int32_t> last((size_t)N, -1);
    for (int32_t i = 0; i < n_objs; ++i) {
        const lq_object& o = objs[i];
        double W;
        bool fg;
        if (!strength(o.law, o.W, S0, &fg, &W, err)) return LQ_EINVAL;
        for (int64_t s : interior[i]) {
            int64_t c[3] = {s % L.n[0], (s / L.n[0]) % L.n[1], s / (L.n[0] * L.n[1])};
            for (int k = 0; k < 3; ++k)
                for (int d = -1; d <= 1; d += 2) {
                    int64_t t = L.nbr(c, k, d);
                    if (t < 0 || g.type[t] == 2 || last[t] == i) continue;
                    last[t] = i;
                    int64_t tc[3] = {t % L.n[0], (t / L.n[0]) % L.n[1], t / (L.n[0] * L.n[1])};
                    if (fg) {
                        double nu[3];
                        surface_normal(o, L, tc[0], tc[1], tc[2], nu);
                        add_fg(row(t), W, nu, S0);
                    } else {
                        double n0[3], q0[5];
                        preferred_director(o, L, tc[0], tc[1], tc[2], n0);
                        q_of(n0, S0, q0);
                        add_nd(row(t), W, q0);
                    }
                }
        }
    }
    for (int64_t i = 0; i < n_recs; ++i) {
        const lq_site_anchor& r = recs[i];
        if (r.site < 0 || r.site >= N || g.type[r.site] == 2) {
            err = "anchoring record outside the simulated sites";
            return LQ_EINVAL;
        }
        double W, n0[3];
        bool fg;
        if (!strength(r.law, r.W, S0, &fg, &W, err)) return LQ_EINVAL;
        if (!normalize(r.n0, n0)) {
            err = "anchoring record director is zero or not finite";
            return LQ_EINVAL;
        }
        if (fg) {
            add_fg(row(r.site), W, n0, S0);
        } else {
            double q0[5];
            q_of(n0, S0, q0);
            add_nd(row(r.site), W, q0);
        }
    }
    // sort the anchored sites
    std::vector<int64_t> order(sites.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return sites[a] < sites[b]; });
    g.anch_site.resize(sites.size());
    g.anch_data.resize(data.size());
    for (size_t i = 0; i < order.size(); ++i) {
        g.anch_site[i] = sites[order[i]];
        std::memcpy(&g.anch_data[ANCH_STRIDE * i], &data[ANCH_STRIDE * order[i]], ANCH_STRIDE * sizeof(double));
        g.type[sites[order[i]]] = 1;
    }
    // neighbour masks
    g.mask.assign((size_t)N, 0);
    g.n_sim = 0;
    for (int64_t z = 0; z < L.n[2]; ++z)
        for (int64_t y = 0; y < L.n[1]; ++y)
            for (int64_t x = 0; x < L.n[0]; ++x) {
                int64_t s = L.idx(x, y, z);
                if (g.type[s] == 2) continue;
                ++g.n_sim;
                int64_t c[3] = {x, y, z};
                uint8_t m = M_SIM;
                for (int k = 0; k < 3; ++k) {
                    int64_t tp = L.nbr(c, k, +1), tm = L.nbr(c, k, -1);
                    if (tp >= 0 && g.type[tp] != 2) m |= (uint8_t)(1u << (2 * k));
                    if (tm >= 0 && g.type[tm] != 2) m |= (uint8_t)(1u << (2 * k + 1));
                }
                if (g.type[s] == 1) m |= M_ANCH;
                g.mask[s] = m;
            }
    return LQ_OK;
}

}  // namespace lq
