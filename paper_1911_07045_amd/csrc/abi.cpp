// Host side of liblqfire: the extern "C" entry points of lqfire.h.
//
// The handle owns the geometry tables on the device (neighbour masks, tile
// flags, anchoring sums) and small scratch for the energy sum.  The caller
// owns every field buffer and the FIRE workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <queue>
#include <string>
#include <vector>

#include "lq_aux.h"
#include "lq_internal.h"

using namespace lq;

struct lq_batch;
static void leave_batch(lq_lattice* lat);

struct lq_lattice {
    lq_batch* batch = nullptr;  // the batch this lattice is a member of, if any
    lq_params p{};
    double S0 = NAN;
    int device = 0;
    hipStream_t stream = nullptr;
    bool l23 = false;
    int64_t N = 0;
    int64_t n_sim = 0;
    // device geometry
    uint8_t* d_mask = nullptr;
    uint8_t* d_tile = nullptr;
    PlaneBits* d_tile_planes = nullptr;
    Chunk* d_chunks = nullptr;
    int32_t* d_first = nullptr;
    int32_t* d_anch_index = nullptr;
    double* d_anch_data = nullptr;
    void* d_anch_force = nullptr;  // K upper triangle and b of each row, in the field's element type
    int n_anch = 0;
    // energy scratch
    double* d_epart = nullptr;
    EnergyOut* d_eout = nullptr;
    uint32_t* d_eticket = nullptr;
    EnergyOut* h_eout = nullptr;  // pinned
    unsigned long long* h_count = nullptr;  // pinned: defect count
    // minimizer binding
    bool bound = false;
    int method = LQ_METHOD_FIRE;
    void* q = nullptr;
    void* v = nullptr;
    void* F = nullptr;
    Bufs<double> b64{};
    Bufs<float> b32{};
    double* d_partials = nullptr;
    FireDev* d_state = nullptr;
    FireDev* h_state = nullptr;  // pinned
    LatDev dev{};
    std::string err;
};

static thread_local std::string g_err;

static int fail(lq_lattice* lat, int code, const std::string& msg) {
    if (lat) lat->err = msg;
    else g_err = msg;
    return code;
}

#define HIPCHK(lat, expr)                                                                 \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(lat, LQ_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    } while (0)

static size_t elem_size(const lq_lattice* lat) { return lat->p.prec == LQ_F64 ? 8 : 4; }

static int check_params(const lq_params* p, std::string& err) {
    if (!p) {
        err = "params is NULL";
        return LQ_EINVAL;
    }
    for (int k = 0; k < 3; ++k) {
        if (p->n[k] < 1 || p->n[k] > (1 << 20)) {
            err = "lattice size out of range";
            return LQ_EINVAL;
        }
        if (p->periodic[k] != 0 && p->periodic[k] != 1) {
            err = "periodic flags must be 0 or 1";
            return LQ_EINVAL;
        }
        if (p->periodic[k] && p->n[k] < 3) {
            err = "a periodic axis needs at least 3 sites";
            return LQ_EINVAL;
        }
    }
    const double N = (double)p->n[0] * (double)p->n[1] * (double)p->n[2];
    if (N > 2147483647.0) {
        err = "more than 2^31 - 1 sites";
        return LQ_EINVAL;
    }
    if (p->prec != LQ_F64 && p->prec != LQ_F32) {
        err = "prec must be LQ_F64 or LQ_F32";
        return LQ_EINVAL;
    }
    // the kernels address one field (5 N values) with 32-bit byte offsets
    if (5.0 * N * (p->prec == LQ_F64 ? 8.0 : 4.0) > 4294967295.0) {
        err = "a field of 5 N values exceeds 2^32 bytes (FP64: N < 107374182, FP32: N < 214748364)";
        return LQ_EINVAL;
    }
    const double c[] = {p->A, p->B, p->C, p->L1, p->L2, p->L3, p->L4, p->L6};
    for (double x : c)
        if (!std::isfinite(x)) {
            err = "non-finite constant";
            return LQ_EINVAL;
        }
    if (p->L6 != 0.0) {
        err = "the L6 term is not built";
        return LQ_EUNSUPPORTED;
    }
    return LQ_OK;
}

static double bulk_S0(const lq_params& p) {
    double disc = p.B * p.B - 24.0 * p.A * p.C;
    if (!(p.C > 0.0) || disc < 0.0) return NAN;
    return (-p.B + std::sqrt(disc)) / (6.0 * p.C);
}

static int check_dev_ptr(lq_lattice* lat, const void* ptr, const char* name) {
    if (!ptr) return fail(lat, LQ_EINVAL, std::string(name) + " is NULL");
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(lat, LQ_EINVAL, std::string(name) + " is not a device pointer");
    }
    if (a.type != hipMemoryTypeDevice || a.device != lat->device)
        return fail(lat, LQ_EINVAL, std::string(name) + " is not device memory of the lattice's device");
    return LQ_OK;
}

// Resident blocks of the fused step kernel on the whole device.
static int64_t resident_blocks(const lq_params& p, int device, bool l23, int wide, bool two = false) {
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n_cu <= 0)
        n_cu = 256;
    return (int64_t)n_cu * step_blocks_per_cu(p.prec, l23, p.L4 != 0.0, wide, two);
}

// The FP64 L2/L3 step kernel holds one wave per SIMD (its registers); held
// to two (a few spilled), it hides more latency but spills.  Measured on one
// GPU: the 128^3 colloid slab 0.153 -> 0.149 ms and the 128^3 bulk box
// 0.131 -> 0.124 ms, but the 256^3 bulk box 0.875 -> 0.902 ms.  So the two-wave
// kernel serves lattices whose one-wave chunks (at one block per compute
// unit) would be shorter than 64 planes.
static bool two_waves_for(const lq_params& p, int device, bool l23, int wide) {
    if (p.prec != LQ_F64 || !l23 || p.L4 != 0.0 || !wide) return false;
    const int64_t TX = tile_x(p.prec, l23, wide), TY = tile_y(p.prec, l23, wide);
    const int64_t ncol = ((p.n[0] + TX - 1) / TX) * ((p.n[1] + TY - 1) / TY);
    return ncol * p.n[2] < 64 * resident_blocks(p, device, l23, wide);
}

// Work of the step kernels.  A block marches one chunk: a run of planes of
// one X x Y column tile.  A plane whose 3 x 3 x 3 neighbourhoods over the
// padded tile are all full bulk sites takes the bulk evaluation; the other
// planes (walls, colloid surfaces) cost about three times as much with L2/L3
// (measured).  When the columns fit in one wave of resident blocks with
// chunks of up to CHUNK_MAX planes, the grid holds one wave: with L2/L3,
// chunks are handed out one at a time to the column whose chunks cost most,
// and every column is cut at equal-cost points (at least 4 planes per
// chunk), so that a step lasts about as long as the average block rather
// than as long as the block that holds a colloid; one-constant lattices,
// whose boundary planes cost little more, get the same equal-length cuts in
// every column, so that neighbouring tiles march the same planes at the same
// time and share their halo planes in L2 (measured faster than cost-balanced
// cuts on the 256^3 multi-colloid box).  Larger lattices take many waves,
// which balance by themselves: one-constant lattices in equal chunks of up
// to 96 planes, L2/L3 lattices with the planes next to a boundary in short
// chunks of their own and the bulk in chunks of up to CHUNK_MAX planes
// (chunk order: at the end of plan_chunks).  Per chunk: whether every
// site of the padded tile over the whole march is a full bulk site, and per
// plane whether that holds for the plane and both its z-neighbours.  LQ_ZC
// (1 .. CHUNK_MAX) forces chunks of that many planes.
struct ChunkPlan {
    std::vector<Chunk> chunks;
    std::vector<uint8_t> bulk;
    std::vector<PlaneBits> planes;
    std::vector<int32_t> first;  // block b marches chunks first[b] .. first[b + 1] - 1
};

static void plan_chunks(const lq_params& p, bool l23, int wide, const std::vector<uint8_t>& mask,
                        int64_t resident, ChunkPlan& out) {
    const int64_t TX = tile_x(p.prec, l23, wide), TY = tile_y(p.prec, l23, wide);
    const int64_t nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int64_t ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, ncol = ntx * nty;
    auto wrap = [](int64_t g, int64_t n, bool per) -> int64_t {
        if (g >= 0 && g < n) return g;
        if (!per) return -1;
        g %= n;
        return g < 0 ? g + n : g;
    };
    // full[c][i]: padded plane z = i - 1 (i = 0 .. nz + 1) of column c is all M_FULL
    const int64_t P = nz + 2;
    std::vector<uint8_t> full((size_t)(ncol * P), 0);
    for (int64_t c = 0; c < ncol; ++c) {
        const int64_t bx = c % ntx, by = c / ntx;
        for (int64_t i = 0; i < P; ++i) {
            const int64_t wz = wrap(i - 1, nz, p.periodic[2]);
            bool ok = wz >= 0;
            for (int64_t y = by * TY - 1; ok && y <= by * TY + TY; ++y) {
                const int64_t wy = wrap(y, ny, p.periodic[1]);
                if (wy < 0) { ok = false; break; }
                for (int64_t x = bx * TX - 1; x <= bx * TX + TX; ++x) {
                    const int64_t wx = wrap(x, nx, p.periodic[0]);
                    if (wx < 0 || mask[wx + nx * (wy + ny * wz)] != M_FULL) { ok = false; break; }
                }
            }
            full[(size_t)(c * P + i)] = ok ? 1 : 0;
        }
    }
    auto F = [&](int64_t c, int64_t i) { return full[(size_t)(c * P + i)] != 0; };
    // cum[c][f]: cost of planes 0 .. f - 1 of column c, a boundary plane
    // costing g bulk planes.  Measured on the 128^3 colloid slab: FP32 best
    // with 3 (2.2 and 3.4 slower by 1.5-2%, 2.6 equal); FP64 with 2.5 (0.1444
    // ms per step, against 0.1486 with 3, 0.1483 with 2 and 0.162 with 1.5).
    const double g = p.prec == LQ_F64 ? 2.5 : 3.0;
    std::vector<double> cum((size_t)(ncol * (nz + 1)), 0.0);
    for (int64_t c = 0; c < ncol; ++c)
        for (int64_t f = 0; f < nz; ++f) {
            const bool bulk = F(c, f) && F(c, f + 1) && F(c, f + 2);
            cum[(size_t)(c * (nz + 1) + f + 1)] = cum[(size_t)(c * (nz + 1) + f)] + (bulk ? 1.0 : g);
        }
    auto total = [&](int64_t c) { return cum[(size_t)(c * (nz + 1) + nz)]; };
    // nonfull[c][i]: padded planes 0 .. i - 1 of column c that are not all M_FULL
    std::vector<int64_t> nonfull((size_t)(ncol * (P + 1)), 0);
    for (int64_t c = 0; c < ncol; ++c)
        for (int64_t i = 0; i < P; ++i)
            nonfull[(size_t)(c * (P + 1) + i + 1)] = nonfull[(size_t)(c * (P + 1) + i)] + (F(c, i) ? 0 : 1);
    // one wave: chunks up to CHUNK_MAX planes; many waves: up to 96 planes
    // (one-constant lattices, and the boundary runs of L2/L3 lattices, below)
    const int64_t zmin = 4;
    const bool one_wave = ncol * ((nz + CHUNK_MAX - 1) / CHUNK_MAX) <= resident;
    const int64_t zmax = one_wave ? CHUNK_MAX : 96;
    const int64_t m_lo = (nz + zmax - 1) / zmax;
    const int64_t m_hi = std::max<int64_t>(m_lo, nz / zmin);
    std::vector<int64_t> m((size_t)ncol, m_lo);
    const char* env = std::getenv("LQ_ZC");
    const int zfix = env ? std::atoi(env) : 0;
    std::vector<std::pair<int64_t, Chunk>> list;  // (rank within the column, chunk)
    typedef std::vector<std::pair<int64_t, Chunk>> Block;
    std::vector<Block> packed;  // non-empty: the blocks of a packed plan
    if (zfix >= 1 && zfix <= CHUNK_MAX) {
        for (int64_t c = 0; c < ncol; ++c)
            for (int64_t z0 = 0, k = 0; z0 < nz; z0 += zfix, ++k)
                list.push_back({k, Chunk{(int32_t)((c % ntx) * TX), (int32_t)((c / ntx) * TY), (int32_t)z0,
                                         (int32_t)std::min<int64_t>(zfix, nz - z0)}});
    } else {
        if (one_wave && !l23) {
            // one-constant lattices: the same cuts in every column (a general
            // plane costs little more than a bulk one here, and aligned chunks
            // let neighbouring tiles share their halo planes in L2)
            const int64_t mu = std::min(std::max(m_lo, resident / std::max<int64_t>(ncol, 1)), m_hi);
            for (int64_t c = 0; c < ncol; ++c) m[(size_t)c] = mu;
        }
        // Cuts of column c into mc chunks: equal plane counts (one-constant
        // lattices) or equal-cost points (L2/L3), every chunk within
        // zlo .. zmax planes.
        auto cuts = [&](int64_t c, int64_t mc) {
            std::vector<int64_t> z(1, 0);
            const double* cc = &cum[(size_t)(c * (nz + 1))];
            for (int64_t k = 1; k <= mc; ++k) {
                const int64_t z0 = z.back();
                int64_t z1 = nz;
                if (k < mc && !l23) {
                    z1 = nz * k / mc;
                } else if (k < mc) {
                    const double target = total(c) * (double)k / (double)mc;
                    const int64_t zlo = std::max<int64_t>(1, std::min<int64_t>(zmin, nz / mc));
                    const int64_t lo_z = std::max(z0 + zlo, nz - zmax * (mc - k));
                    const int64_t hi_z = std::min(z0 + zmax, nz - zlo * (mc - k));
                    z1 = lo_z;
                    while (z1 < hi_z && cc[z1] < target) ++z1;
                    if (z1 > lo_z && cc[z1] - target > target - cc[z1 - 1]) --z1;
                }
                z.push_back(z1);
            }
            return z;
        };
        // Time of one chunk in plane units: its planes (a boundary plane g),
        // 13% more where the chunk holds any boundary plane (its march reads
        // masks and anchoring indices for every plane), and two planes for
        // the halo planes and the pipeline's start (measured on the 128^3
        // colloid slab, FP32 and FP64).
        auto chunk_cost = [&](int64_t c, int64_t z0, int64_t z1) {
            const int64_t* nf = &nonfull[(size_t)(c * (P + 1))];
            const bool all = nf[z1 + 2] - nf[z0] == 0;
            const double* cc = &cum[(size_t)(c * (nz + 1))];
            return (cc[z1] - cc[z0]) * (all ? 1.0 : 1.13) + 2.0;
        };
        auto worst = [&](int64_t c, int64_t mc) {
            const std::vector<int64_t> z = cuts(c, mc);
            double w = 0.0;
            for (size_t k = 1; k < z.size(); ++k) w = std::max(w, chunk_cost(c, z[k - 1], z[k]));
            return w;
        };
        // L2/L3: one more chunk at a time to the column whose costliest chunk
        // costs most, until the chunks fill one wave of resident blocks
        std::priority_queue<std::pair<double, int64_t>> heavy;
        if (one_wave && l23)
            for (int64_t c = 0; c < ncol; ++c) heavy.push({worst(c, m_lo), c});
        for (int64_t blocks = ncol * m_lo; one_wave && l23 && blocks < resident && !heavy.empty();) {
            const int64_t c = heavy.top().second;
            heavy.pop();
            if (m[(size_t)c] >= m_hi) continue;
            ++m[(size_t)c];
            ++blocks;
            heavy.push({worst(c, m[(size_t)c]), c});
        }
        // Many waves with L2/L3: each run of planes whose neighbourhoods reach
        // a boundary marches in chunks of its own (widened to WALL_Z planes,
        // up to zmax), the bulk between the runs in chunks of up to BULK_Z
        // planes, so that the bulk planes take no boundary chunk's per-plane
        // mask and anchoring reads.  On the 512^3 patterned wall, ms per step:
        // equal-cost cuts of up to 96 planes 3.757; wall chunks of 8 planes
        // with bulk chunks of up to 128 planes 3.636, 168 3.615, 256 3.597;
        // wall chunks of 16 or 32 planes (bulk 128) 3.656 and 3.681, of 4
        // planes 3.624 (bulk 128) and 3.607 (bulk 168).
        const int64_t WALL_Z = 8, BULK_Z = CHUNK_MAX;
        auto wall_cuts = [&](int64_t c) {
            const int64_t W = std::min<int64_t>(WALL_Z, nz);
            std::vector<std::pair<int64_t, int64_t>> reg;
            for (int64_t f = 0; f < nz;) {
                if (F(c, f) && F(c, f + 1) && F(c, f + 2)) { ++f; continue; }
                int64_t e = f;
                while (e < nz && !(F(c, e) && F(c, e + 1) && F(c, e + 2))) ++e;
                int64_t a = f;
                if (e - a < W) {
                    a = std::max<int64_t>(0, a - (W - (e - a)) / 2);
                    e = std::min<int64_t>(nz, a + W);
                    a = std::max<int64_t>(0, e - W);
                }
                if (!reg.empty() && a <= reg.back().second + zmin) reg.back().second = std::max(reg.back().second, e);
                else reg.push_back({a, e});
                f = e;
            }
            if (!reg.empty() && reg.front().first <= zmin) reg.front().first = 0;
            if (!reg.empty() && nz - reg.back().second <= zmin) reg.back().second = nz;
            std::vector<int64_t> z(1, 0);
            auto span = [&](int64_t a, int64_t b, int64_t zm) {
                const int64_t n = (b - a + zm - 1) / zm;
                for (int64_t k = 1; k <= n; ++k) z.push_back(a + (b - a) * k / n);
            };
            int64_t at = 0;
            for (const auto& r : reg) {
                if (r.first > at) span(at, r.first, BULK_Z);
                span(r.first, r.second, zmax);
                at = r.second;
            }
            if (at < nz) span(at, nz, BULK_Z);
            return z;
        };
        const bool by_walls = !one_wave && l23;
        double worst_chunk = 0.0;
        for (int64_t c = 0; c < ncol; ++c) {
            const std::vector<int64_t> z = by_walls ? wall_cuts(c) : cuts(c, m[(size_t)c]);
            for (size_t k = 1; k < z.size(); ++k) {
                list.push_back({(int64_t)k - 1, Chunk{(int32_t)((c % ntx) * TX), (int32_t)((c / ntx) * TY),
                                                      (int32_t)z[k - 1], (int32_t)(z[k] - z[k - 1])}});
                worst_chunk = std::max(worst_chunk, chunk_cost(c, z[k - 1], z[k]));
            }
        }
        // Packed plan (one wave, FP64 L2/L3; the step kernels of the other
        // plans march one chunk per block): with few columns per resident
        // block (64 FP64 columns of the 128^3 slab for 256 blocks) whole
        // chunks per column cannot balance the columns' costs.  Each column is cut from
        // the bottom into chunks of cost at most M, the chunks are paired
        // largest with smallest while a pair stays within M, and a block
        // marches its pair one chunk after the other; M is the least value
        // (bisection) whose blocks fit in one wave.  Taken when it lowers the
        // costliest block by 3% or more.
        auto pack = [&](double M, std::vector<Block>& blk) {
            blk.clear();
            std::vector<std::pair<double, std::pair<int64_t, Chunk>>> pieces;
            for (int64_t c = 0; c < ncol; ++c) {
                for (int64_t z0 = 0, k = 0; z0 < nz; ++k) {
                    int64_t z1 = std::min(nz, z0 + zmin);
                    while (z1 < nz && z1 - z0 < zmax && chunk_cost(c, z0, z1 + 1) <= M) ++z1;
                    // no last chunk below zmin planes
                    if (z1 < nz && nz - z1 < zmin) z1 = nz - z0 >= 2 * zmin ? nz - zmin : nz;
                    pieces.push_back({chunk_cost(c, z0, z1),
                                      {k, Chunk{(int32_t)((c % ntx) * TX), (int32_t)((c / ntx) * TY), (int32_t)z0,
                                                (int32_t)(z1 - z0)}}});
                    z0 = z1;
                }
            }
            std::stable_sort(pieces.begin(), pieces.end(),
                             [](const std::pair<double, std::pair<int64_t, Chunk>>& a,
                                const std::pair<double, std::pair<int64_t, Chunk>>& b) { return a.first > b.first; });
            for (size_t i = 0, j = pieces.size(); i < j; ++i) {
                blk.push_back(Block(1, pieces[i].second));
                if (j - 1 > i && pieces[i].first + pieces[j - 1].first <= M) blk.back().push_back(pieces[--j].second);
            }
            return (int64_t)blk.size();
        };
        if (one_wave && l23 && p.prec == LQ_F64 && zfix == 0) {
            std::vector<Block> trial;
            double lo = 0.0, hi = worst_chunk;
            for (int it = 0; it < 40; ++it) {
                const double M = 0.5 * (lo + hi);
                if (pack(M, trial) <= resident) hi = M;
                else lo = M;
            }
            if (hi < 0.97 * worst_chunk && pack(hi, trial) <= resident) packed.swap(trial);
        }
    }
    // One wave: by rank within the column, then tile row and column (every
    // block runs at once; neighbouring tiles march the same planes together).
    // Many waves: the step kernel hands each XCD a contiguous eighth of the
    // list, so the columns are split into eight groups of neighbouring
    // columns and each group is listed by rank, then column: every XCD then
    // gets its share of the heavier wall chunks (by rank alone, the first and
    // last eighths held all of them), and neighbouring columns still march
    // the same planes together.
    // A block marches one chunk, or (packed plans) two chunks one after the
    // other; it is ordered by its first chunk.
    typedef std::vector<std::pair<int64_t, Chunk>> Block;
    std::vector<Block> blocks;
    for (const auto& e : list) blocks.push_back(Block(1, e));
    if (!packed.empty()) blocks.swap(packed);
    const int64_t gsize = one_wave ? ncol : (ncol + 7) / 8;
    std::stable_sort(blocks.begin(), blocks.end(), [&](const Block& A, const Block& B) {
        const std::pair<int64_t, Chunk>& a = A.front();
        const std::pair<int64_t, Chunk>& b = B.front();
        const int64_t ca = a.second.x0 / TX + ntx * (a.second.y0 / TY);
        const int64_t cb = b.second.x0 / TX + ntx * (b.second.y0 / TY);
        if (ca / gsize != cb / gsize) return ca / gsize < cb / gsize;
        return a.first < b.first;
    });
    out.chunks.clear();
    out.bulk.clear();
    out.planes.clear();
    out.first.assign(1, 0);
    for (const Block& blk : blocks) {
      for (const auto& e : blk) {
        const Chunk& ch = e.second;
        const int64_t c = ch.x0 / TX + ntx * (ch.y0 / TY);
        bool all = true;
        for (int64_t i = ch.z0; i <= ch.z0 + ch.zc + 1; ++i) all = all && F(c, i);
        PlaneBits bits{};
        for (int64_t f = 0; f < std::min<int64_t>(ch.zc, CHUNK_MAX); ++f)
            if (F(c, ch.z0 + f) && F(c, ch.z0 + f + 1) && F(c, ch.z0 + f + 2))
                bits.w[f / 64] |= (uint64_t)1 << (f % 64);
        out.chunks.push_back(ch);
        out.bulk.push_back(all ? 1 : 0);
        out.planes.push_back(bits);
      }
      out.first.push_back((int32_t)out.chunks.size());
    }
}

static void free_geometry(lq_lattice* lat) {
    if (lat->d_mask) (void)hipFree(lat->d_mask);
    if (lat->d_tile) (void)hipFree(lat->d_tile);
    if (lat->d_tile_planes) (void)hipFree(lat->d_tile_planes);
    if (lat->d_chunks) (void)hipFree(lat->d_chunks);
    if (lat->d_first) (void)hipFree(lat->d_first);
    if (lat->d_anch_index) (void)hipFree(lat->d_anch_index);
    if (lat->d_anch_data) (void)hipFree(lat->d_anch_data);
    if (lat->d_anch_force) (void)hipFree(lat->d_anch_force);
    lat->d_mask = lat->d_tile = nullptr;
    lat->d_tile_planes = nullptr;
    lat->d_anch_index = nullptr;
    lat->d_anch_data = nullptr;
    lat->d_anch_force = nullptr;
    lat->d_chunks = nullptr;
    lat->d_first = nullptr;
}

// Uploads a rasterized geometry and refreshes the device view.
static int upload_geometry(lq_lattice* lat, const Geometry& g) {
    HIPCHK(lat, hipSetDevice(lat->device));
    HIPCHK(lat, hipStreamSynchronize(lat->stream));
    free_geometry(lat);
    const lq_params& p = lat->p;
    LatDev& d = lat->dev;
    d.nx = (int)p.n[0]; d.ny = (int)p.n[1]; d.nz = (int)p.n[2];
    for (int k = 0; k < 3; ++k) d.per[k] = p.periodic[k];
    d.N = lat->N;
    d.A = p.A; d.B = p.B; d.C = p.C; d.L1 = p.L1; d.L2 = p.L2; d.L3 = p.L3; d.L4 = p.L4;
    d.wide = tile_wide_for(p.n[0], p.prec, lat->l23);
    ChunkPlan plan;
    d.two_waves = two_waves_for(p, lat->device, lat->l23, d.wide) ? 1 : 0;
    plan_chunks(p, lat->l23, d.wide, g.mask, resident_blocks(p, lat->device, lat->l23, d.wide, d.two_waves != 0),
                plan);
    d.nchunks = (int)plan.chunks.size();
    d.nblocks = (int)plan.first.size() - 1;
    HIPCHK(lat, hipMalloc(&lat->d_first, plan.first.size() * sizeof(int32_t)));
    HIPCHK(lat, hipMemcpy(lat->d_first, plan.first.data(), plan.first.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
    const std::vector<uint8_t>& tiles = plan.bulk;
    const std::vector<PlaneBits>& tile_planes = plan.planes;
    HIPCHK(lat, hipMalloc(&lat->d_chunks, plan.chunks.size() * sizeof(Chunk)));
    HIPCHK(lat, hipMemcpy(lat->d_chunks, plan.chunks.data(), plan.chunks.size() * sizeof(Chunk),
                          hipMemcpyHostToDevice));
    HIPCHK(lat, hipMalloc(&lat->d_mask, (size_t)lat->N));
    HIPCHK(lat, hipMemcpy(lat->d_mask, g.mask.data(), (size_t)lat->N, hipMemcpyHostToDevice));
    HIPCHK(lat, hipMalloc(&lat->d_tile, tiles.size()));
    HIPCHK(lat, hipMemcpy(lat->d_tile, tiles.data(), tiles.size(), hipMemcpyHostToDevice));
    HIPCHK(lat, hipMalloc(&lat->d_tile_planes, tile_planes.size() * sizeof(PlaneBits)));
    HIPCHK(lat, hipMemcpy(lat->d_tile_planes, tile_planes.data(), tile_planes.size() * sizeof(PlaneBits),
                          hipMemcpyHostToDevice));
    lat->n_anch = (int)g.anch_site.size();
    if (lat->n_anch > 0) {
        // dense per-site row index (1-based; 0 = no anchoring)
        std::vector<int32_t> idx((size_t)lat->N, 0);
        for (size_t i = 0; i < g.anch_site.size(); ++i) idx[(size_t)g.anch_site[i]] = (int32_t)i + 1;
        HIPCHK(lat, hipMalloc(&lat->d_anch_index, idx.size() * sizeof(int32_t)));
        HIPCHK(lat, hipMemcpy(lat->d_anch_index, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(lat, hipMalloc(&lat->d_anch_data, g.anch_data.size() * sizeof(double)));
        HIPCHK(lat, hipMemcpy(lat->d_anch_data, g.anch_data.data(), g.anch_data.size() * sizeof(double),
                              hipMemcpyHostToDevice));
        // the force needs K and b only: ANCH_FSTRIDE values per row, rounded
        // to the field's element type once here
        const size_t rows = g.anch_site.size();
        if (lat->p.prec == LQ_F64) {
            std::vector<double> f(rows * ANCH_FSTRIDE);
            for (size_t i = 0; i < rows; ++i)
                for (int k = 0; k < ANCH_FSTRIDE; ++k) f[i * ANCH_FSTRIDE + k] = g.anch_data[i * ANCH_STRIDE + k];
            HIPCHK(lat, hipMalloc(&lat->d_anch_force, f.size() * sizeof(double)));
            HIPCHK(lat, hipMemcpy(lat->d_anch_force, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice));
        } else {
            std::vector<float> f(rows * ANCH_FSTRIDE);
            for (size_t i = 0; i < rows; ++i)
                for (int k = 0; k < ANCH_FSTRIDE; ++k)
                    f[i * ANCH_FSTRIDE + k] = (float)g.anch_data[i * ANCH_STRIDE + k];
            HIPCHK(lat, hipMalloc(&lat->d_anch_force, f.size() * sizeof(float)));
            HIPCHK(lat, hipMemcpy(lat->d_anch_force, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
        }
    }
    d.mask = lat->d_mask;
    d.chunks = lat->d_chunks;
    d.first = lat->d_first;
    d.tile_bulk = lat->d_tile;
    d.tile_planes = lat->d_tile_planes;
    d.n_anch = lat->n_anch;
    d.anch_index = lat->d_anch_index;
    d.anch_data = lat->d_anch_data;
    d.anch_force = lat->d_anch_force;
    lat->n_sim = g.n_sim;
    lat->bound = false;
    return LQ_OK;
}

extern "C" {

int lq_lattice_create(const lq_params* p, void* stream, lq_lattice** out) {
    std::string err;
    if (!out) return fail(nullptr, LQ_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(p, err);
    if (rc != LQ_OK) return fail(nullptr, rc, err);
    lq_lattice* lat = new lq_lattice();
    lat->p = *p;
    lat->S0 = bulk_S0(*p);
    lat->stream = (hipStream_t)stream;
    lat->l23 = p->L2 != 0.0 || p->L3 != 0.0 || p->L4 != 0.0;
    lat->N = p->n[0] * p->n[1] * p->n[2];
    hipError_t e = hipGetDevice(&lat->device);
    if (e != hipSuccess) {
        delete lat;
        return fail(nullptr, LQ_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    Geometry g;
    rc = rasterize(lat->p, lat->S0, nullptr, 0, nullptr, 0, nullptr, 0, g, err);
    if (rc == LQ_OK) rc = upload_geometry(lat, g);
    if (rc == LQ_OK) {
        const int64_t nb = std::max<int64_t>(n_energy_blocks(lat->dev), 1);
        if (hipMalloc(&lat->d_epart, (size_t)nb * 4 * sizeof(double)) != hipSuccess ||
            hipMalloc(&lat->d_eout, sizeof(EnergyOut)) != hipSuccess ||
            hipMalloc(&lat->d_eticket, 256) != hipSuccess ||
            hipHostMalloc(&lat->h_eout, sizeof(EnergyOut), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&lat->h_state, sizeof(FireDev), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&lat->h_count, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
            hipMemset(lat->d_eticket, 0, 256) != hipSuccess) {
            (void)hipGetLastError();
            err = "device allocation failed";
            rc = LQ_ENOMEM;
        }
    } else if (err.empty()) {
        err = lat->err;
    }
    if (rc != LQ_OK) {
        lq_lattice_destroy(lat);
        return fail(nullptr, rc, err);
    }
    *out = lat;
    return LQ_OK;
}

int lq_lattice_destroy(lq_lattice* lat) {
    if (!lat) return LQ_OK;
    leave_batch(lat);
    (void)hipSetDevice(lat->device);
    (void)hipStreamSynchronize(lat->stream);
    free_geometry(lat);
    if (lat->d_epart) (void)hipFree(lat->d_epart);
    if (lat->d_eout) (void)hipFree(lat->d_eout);
    if (lat->d_eticket) (void)hipFree(lat->d_eticket);
    if (lat->h_eout) (void)hipHostFree(lat->h_eout);
    if (lat->h_count) (void)hipHostFree(lat->h_count);
    if (lat->h_state) (void)hipHostFree(lat->h_state);
    delete lat;
    return LQ_OK;
}

double lq_bulk_S0(const lq_lattice* lat) { return lat ? lat->S0 : NAN; }

int lq_rasterize(const lq_params* p, const lq_object* objs, int32_t n_objs, const lq_site_anchor* recs,
                 int64_t n_recs, const int64_t* object_sites, int64_t n_object_sites, uint8_t* types,
                 int64_t* n_anchored, int64_t* anch_site, double* anch_data, int64_t cap) {
    std::string err;
    int rc = check_params(p, err);
    if (rc != LQ_OK) return fail(nullptr, rc, err);
    if (cap < 0 || (cap > 0 && (!anch_site || !anch_data)))
        return fail(nullptr, LQ_EINVAL, "bad output arrays");
    Geometry g;
    rc = rasterize(*p, bulk_S0(*p), objs, n_objs, recs, n_recs, object_sites, n_object_sites, g, err);
    if (rc != LQ_OK) return fail(nullptr, rc, err);
    if (types) std::memcpy(types, g.type.data(), g.type.size());
    if (n_anchored) *n_anchored = (int64_t)g.anch_site.size();
    const int64_t n = std::min<int64_t>(cap, (int64_t)g.anch_site.size());
    for (int64_t i = 0; i < n; ++i) {
        anch_site[i] = g.anch_site[i];
        std::memcpy(anch_data + ANCH_STRIDE * i, &g.anch_data[ANCH_STRIDE * i], ANCH_STRIDE * sizeof(double));
    }
    return LQ_OK;
}

int lq_step_plan(const lq_params* p, const lq_object* objs, int32_t n_objs, int64_t resident,
                 int32_t* chunks, uint8_t* bulk, int32_t* block, int64_t cap, int64_t* n_chunks,
                 int32_t* tile_nx, int32_t* tile_ny) {
    std::string err;
    int rc = check_params(p, err);
    if (rc != LQ_OK) return fail(nullptr, rc, err);
    if (resident <= 0) return fail(nullptr, LQ_EINVAL, "resident must be positive");
    if (cap < 0 || (cap > 0 && (!chunks || !bulk))) return fail(nullptr, LQ_EINVAL, "bad output arrays");
    Geometry g;
    rc = rasterize(*p, bulk_S0(*p), objs, n_objs, nullptr, 0, nullptr, 0, g, err);
    if (rc != LQ_OK) return fail(nullptr, rc, err);
    const bool l23 = p->L2 != 0.0 || p->L3 != 0.0 || p->L4 != 0.0;
    const int wide = tile_wide_for(p->n[0], p->prec, l23);
    ChunkPlan plan;
    plan_chunks(*p, l23, wide, g.mask, resident, plan);
    const int64_t n = (int64_t)plan.chunks.size();
    for (int64_t i = 0; i < std::min(n, cap); ++i) {
        const Chunk& c = plan.chunks[(size_t)i];
        chunks[4 * i + 0] = c.x0;
        chunks[4 * i + 1] = c.y0;
        chunks[4 * i + 2] = c.z0;
        chunks[4 * i + 3] = c.zc;
        bulk[i] = plan.bulk[(size_t)i];
    }
    if (block)
        for (size_t b = 0; b + 1 < plan.first.size(); ++b)
            for (int32_t i = plan.first[b]; i < plan.first[b + 1] && (int64_t)i < cap; ++i) block[i] = (int32_t)b;
    if (n_chunks) *n_chunks = n;
    if (tile_nx) *tile_nx = lq::tile_x(p->prec, l23, wide);
    if (tile_ny) *tile_ny = lq::tile_y(p->prec, l23, wide);
    return LQ_OK;
}

int lq_set_boundaries(lq_lattice* lat, const lq_object* objs, int32_t n_objs, const lq_site_anchor* recs,
                      int64_t n_recs, const int64_t* object_sites, int64_t n_object_sites) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    std::string err;
    Geometry g;
    int rc = rasterize(lat->p, lat->S0, objs, n_objs, recs, n_recs, object_sites, n_object_sites, g, err);
    if (rc != LQ_OK) return fail(lat, rc, err);
    // the step kernels address the anchoring rows (ANCH_FSTRIDE values of the
    // field's type each) with 32-bit byte offsets
    if ((uint64_t)g.anch_site.size() * (uint64_t)(ANCH_FSTRIDE * elem_size(lat)) > 0xFFFFFFFFull)
        return fail(lat, LQ_EINVAL, "too many anchored sites (at most 53687091 in FP32, 26843545 in FP64)");
    return upload_geometry(lat, g);
}

int lq_set_field(lq_lattice* lat, const double* h, const double* chi, int32_t n_fields) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    if (n_fields < 0 || (n_fields > 0 && (!h || !chi))) return fail(lat, LQ_EINVAL, "bad field arrays");
    // hf = sum chi/3 h h^T; the force on q is +P^T hf
    double hf[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int32_t f = 0; f < n_fields; ++f) {
        const double* v = h + 3 * (int64_t)f;
        if (!std::isfinite(chi[f]) || !std::isfinite(v[0]) || !std::isfinite(v[1]) || !std::isfinite(v[2]))
            return fail(lat, LQ_EINVAL, "field is not finite");
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) hf[a][b] += chi[f] / 3.0 * v[a] * v[b];
    }
    double* e = lat->dev.ext;
    e[0] = hf[0][0] - hf[2][2];
    e[1] = hf[0][1] + hf[1][0];
    e[2] = hf[0][2] + hf[2][0];
    e[3] = hf[1][1] - hf[2][2];
    e[4] = hf[1][2] + hf[2][1];
    lat->bound = false;
    return LQ_OK;
}

int lq_set_uniaxial(lq_lattice* lat, const double* directors, double S, void* q) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    if (!std::isfinite(S)) return fail(lat, LQ_EINVAL, "S is not finite");
    int rc = check_dev_ptr(lat, directors, "directors");
    if (rc == LQ_OK) rc = check_dev_ptr(lat, q, "q");
    if (rc != LQ_OK) return rc;
    HIPCHK(lat, hipSetDevice(lat->device));
    rc = launch_uniaxial(lat->dev, lat->p.prec, directors, S, q, lat->stream);
    if (rc != LQ_OK) return fail(lat, rc, "kernel launch failed");
    return LQ_OK;
}

int lq_compute_forces(lq_lattice* lat, const void* q, void* F) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    int rc = check_dev_ptr(lat, q, "q");
    if (rc == LQ_OK) rc = check_dev_ptr(lat, F, "F");
    if (rc != LQ_OK) return rc;
    if (q == F) return fail(lat, LQ_EINVAL, "q and F must not alias");
    HIPCHK(lat, hipSetDevice(lat->device));
    rc = launch_forces(lat->dev, lat->l23, lat->p.prec, q, F, lat->stream);
    if (rc != LQ_OK) return fail(lat, rc, "kernel launch failed");
    return LQ_OK;
}

int lq_energy(lq_lattice* lat, const void* q, lq_energy_terms* out) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    if (!out) return fail(lat, LQ_EINVAL, "out is NULL");
    int rc = check_dev_ptr(lat, q, "q");
    if (rc != LQ_OK) return rc;
    HIPCHK(lat, hipSetDevice(lat->device));
    rc = launch_energy(lat->dev, lat->l23, lat->p.prec, q, lat->d_epart, lat->d_eout, lat->d_eticket,
                       lat->stream);
    if (rc != LQ_OK) return fail(lat, rc, "kernel launch failed");
    HIPCHK(lat, hipMemcpyAsync(lat->h_eout, lat->d_eout, sizeof(EnergyOut), hipMemcpyDeviceToHost, lat->stream));
    HIPCHK(lat, hipStreamSynchronize(lat->stream));
    out->bulk = lat->h_eout->bulk;
    out->elastic = lat->h_eout->elastic;
    out->anchoring = lat->h_eout->anch;
    out->external = lat->h_eout->ext;
    out->total = out->bulk + out->elastic + out->anchoring + out->external;
    out->n_sim = lat->n_sim;
    return LQ_OK;
}

int lq_director_field(lq_lattice* lat, const void* q, void* dirs, void* lambda_max, uint8_t* defect,
                      double threshold, int64_t* n_defects) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    if (!std::isfinite(threshold)) return fail(lat, LQ_EINVAL, "threshold is not finite");
    int rc = check_dev_ptr(lat, q, "q");
    if (rc == LQ_OK && dirs) rc = check_dev_ptr(lat, dirs, "dirs");
    if (rc == LQ_OK && lambda_max) rc = check_dev_ptr(lat, lambda_max, "lambda_max");
    if (rc == LQ_OK && defect) rc = check_dev_ptr(lat, defect, "defect");
    if (rc != LQ_OK) return rc;
    if (q == dirs || q == lambda_max || (dirs && dirs == lambda_max))
        return fail(lat, LQ_EINVAL, "outputs must not alias q or each other");
    HIPCHK(lat, hipSetDevice(lat->device));
    // the defect counter sits in the energy kernel's ticket block, past the ticket
    unsigned long long* d_count = n_defects ? (unsigned long long*)((char*)lat->d_eticket + 128) : nullptr;
    rc = launch_directors(lat->dev, lat->p.prec, q, dirs, lambda_max, defect, threshold, d_count, lat->stream);
    if (rc != LQ_OK) return fail(lat, rc, "kernel launch failed");
    if (n_defects) {
        HIPCHK(lat, hipMemcpyAsync(lat->h_count, d_count, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                   lat->stream));
        HIPCHK(lat, hipStreamSynchronize(lat->stream));
        *n_defects = (int64_t)*lat->h_count;
    }
    return LQ_OK;
}

static int64_t partial_slots(const lq_lattice* lat) {
    return std::max<int64_t>(n_step_blocks(lat->dev), n_energy_blocks(lat->dev));
}

static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Workspace: the second buffer of q, v and F; two slots of block partials
// (step k writes slot k & 1 while step k + 1 reads it); the controller
// state st[2] and its DcCtl word.
static int64_t partials_bytes(const lq_lattice* lat) {
    return align256(2 * partial_slots(lat) * 4 * (int64_t)sizeof(double));
}

int64_t lq_workspace_bytes(const lq_lattice* lat) {
    if (!lat) return -1;
    const int64_t field = align256(5 * lat->N * (int64_t)elem_size(lat));
    return 3 * field + partials_bytes(lat) + align256(2 * (int64_t)sizeof(FireDev) + (int64_t)sizeof(DcCtl));
}

static int check_fire_params(lq_lattice* lat, const lq_fire_params* fp) {
    if (!fp) return fail(lat, LQ_EINVAL, "FIRE params is NULL");
    const double v[] = {fp->dt0, fp->dt_max, fp->alpha0, fp->f_inc, fp->f_dec, fp->f_alpha, fp->force_tol};
    for (double x : v)
        if (!std::isfinite(x)) return fail(lat, LQ_EINVAL, "non-finite FIRE parameter");
    if (!(fp->dt0 > 0.0) || !(fp->dt_max > 0.0) || fp->alpha0 < 0.0 || fp->alpha0 > 1.0 ||
        !(fp->f_inc >= 1.0) || !(fp->f_dec > 0.0) || !(fp->f_dec <= 1.0) || !(fp->f_alpha > 0.0) ||
        fp->f_alpha > 1.0 || fp->n_min < 0 || fp->force_tol < 0.0 || fp->max_steps < 0)
        return fail(lat, LQ_EINVAL, "FIRE parameter out of range");
    return LQ_OK;
}

// Checks and binds q, v, F and the workspace (ping-pong buffers, partials,
// device state).  Leaves the lattice unbound.
static int bind_buffers(lq_lattice* lat, void* q, void* v, void* F, void* workspace, int64_t workspace_bytes) {
    int rc = check_dev_ptr(lat, q, "q");
    if (rc == LQ_OK) rc = check_dev_ptr(lat, v, "v");
    if (rc == LQ_OK) rc = check_dev_ptr(lat, F, "F");
    if (rc == LQ_OK) rc = check_dev_ptr(lat, workspace, "workspace");
    if (rc != LQ_OK) return rc;
    if (q == v || q == F || v == F) return fail(lat, LQ_EINVAL, "q, v and F must be distinct buffers");
    if (workspace_bytes < lq_workspace_bytes(lat))
        return fail(lat, LQ_ENOMEM, "workspace smaller than lq_workspace_bytes()");
    if (((uintptr_t)workspace & 255) != 0) return fail(lat, LQ_EINVAL, "workspace must be 256-byte aligned");
    const int64_t field = align256(5 * lat->N * (int64_t)elem_size(lat));
    char* ws = (char*)workspace;
    void* q1 = ws;
    void* v1 = ws + field;
    void* F1 = ws + 2 * field;
    lat->d_partials = (double*)(ws + 3 * field);
    lat->d_state = (FireDev*)(ws + 3 * field + partials_bytes(lat));
    lat->q = q;
    lat->v = v;
    lat->F = F;
    lat->b64 = Bufs<double>{{(double*)q, (double*)q1}, {(double*)v, (double*)v1}, {(double*)F, (double*)F1}};
    lat->b32 = Bufs<float>{{(float*)q, (float*)q1}, {(float*)v, (float*)v1}, {(float*)F, (float*)F1}};
    return LQ_OK;
}

// Uploads the host controller, runs the initial reduction (with v, or
// without when v_red is NULL) and binds the lattice.
static int start_controller(lq_lattice* lat, FireDev& s, const void* v_red) {
    HIPCHK(lat, hipMemcpyAsync(lat->d_state, &s, sizeof(FireDev), hipMemcpyHostToDevice, lat->stream));
    int rc = launch_fire_init_reduce(lat->dev, lat->p.prec, lat->F, v_red, lat->d_partials, lat->d_state,
                                     lat->stream);
    if (rc != LQ_OK) return fail(lat, rc, "kernel launch failed");
    HIPCHK(lat, hipMemcpyAsync(lat->h_state, lat->d_state, sizeof(FireDev), hipMemcpyDeviceToHost, lat->stream));
    HIPCHK(lat, hipStreamSynchronize(lat->stream));
    lat->bound = true;
    if (lat->h_state->status == LQ_NONFINITE) return fail(lat, LQ_ENONFINITE, "initial forces are not finite");
    return LQ_OK;
}

int lq_fire_init(lq_lattice* lat, const lq_fire_params* fp, void* q, void* v, void* F, void* workspace,
                 int64_t workspace_bytes, const lq_fire_report* resume) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    lat->bound = false;
    int rc = check_fire_params(lat, fp);
    if (rc != LQ_OK) return rc;
    if (resume) {
        if (!(resume->dt > 0.0) || !std::isfinite(resume->dt) || !(resume->alpha >= 0.0) ||
            !(resume->alpha <= 1.0) || resume->step < 0 || resume->n_pos < 0 || resume->restarts < 0)
            return fail(lat, LQ_EINVAL, "bad resume state");
    }
    HIPCHK(lat, hipSetDevice(lat->device));
    rc = bind_buffers(lat, q, v, F, workspace, workspace_bytes);
    if (rc != LQ_OK) return rc;
    lat->method = LQ_METHOD_FIRE;
    rc = launch_forces(lat->dev, lat->l23, lat->p.prec, q, F, lat->stream);
    if (rc == LQ_OK && !resume) rc = launch_fill_zero(v, 5 * lat->N * (int64_t)elem_size(lat), lat->stream);
    if (rc != LQ_OK) return fail(lat, rc, "kernel launch failed");
    FireDev& s = *lat->h_state;
    std::memset(&s, 0, sizeof(FireDev));
    s.dt = resume ? resume->dt : fp->dt0;
    s.alpha = resume ? resume->alpha : fp->alpha0;
    s.c_v = 1.0;
    s.c_F = 0.0;
    s.n_pos = resume ? resume->n_pos : 0;
    s.step = resume ? resume->step : 0;
    s.restarts = resume ? resume->restarts : 0;
    s.stop_at = s.step;
    s.cur = 0;
    s.done = 0;
    s.status = LQ_RUNNING;
    s.init_pending = 1;
    s.dt_max = fp->dt_max;
    s.alpha0 = fp->alpha0;
    s.f_inc = fp->f_inc;
    s.f_dec = fp->f_dec;
    s.f_alpha = fp->f_alpha;
    s.tol = fp->force_tol;
    s.n_min = fp->n_min;
    s.max_steps = fp->max_steps;
    s.ticket = 0;
    s.method = LQ_METHOD_FIRE;
    return start_controller(lat, s, v);
}

int lq_descent_init(lq_lattice* lat, const lq_descent_params* dp, void* q, void* v, void* F, void* workspace,
                    int64_t workspace_bytes, const lq_fire_report* resume) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    lat->bound = false;
    if (!dp) return fail(lat, LQ_EINVAL, "descent params is NULL");
    if (dp->method != LQ_METHOD_GD && dp->method != LQ_METHOD_NESTEROV)
        return fail(lat, LQ_EINVAL, "method must be LQ_METHOD_GD or LQ_METHOD_NESTEROV");
    if (!std::isfinite(dp->dt) || !(dp->dt > 0.0) || !std::isfinite(dp->force_tol) || dp->force_tol < 0.0 ||
        dp->max_steps < 0)
        return fail(lat, LQ_EINVAL, "descent parameter out of range");
    const bool nag = dp->method == LQ_METHOD_NESTEROV;
    if (nag && !(dp->momentum >= 0.0 && dp->momentum < 1.0))
        return fail(lat, LQ_EINVAL, "Nesterov momentum must lie in [0, 1)");
    if (resume && resume->step < 0) return fail(lat, LQ_EINVAL, "bad resume state");
    HIPCHK(lat, hipSetDevice(lat->device));
    int rc = bind_buffers(lat, q, v, F, workspace, workspace_bytes);
    if (rc != LQ_OK) return rc;
    lat->method = dp->method;
    if (nag && resume) {
        // force at the look-ahead point, built in the spare q buffer
        void* y = lat->p.prec == LQ_F64 ? (void*)lat->b64.q[1] : (void*)lat->b32.q[1];
        rc = launch_lookahead(lat->dev, lat->p.prec, q, v, dp->momentum, y, lat->stream);
        if (rc == LQ_OK) rc = launch_forces(lat->dev, lat->l23, lat->p.prec, y, F, lat->stream);
    } else {
        rc = launch_forces(lat->dev, lat->l23, lat->p.prec, q, F, lat->stream);
        if (rc == LQ_OK && nag) rc = launch_fill_zero(v, 5 * lat->N * (int64_t)elem_size(lat), lat->stream);
    }
    if (rc != LQ_OK) return fail(lat, rc, "kernel launch failed");
    FireDev& s = *lat->h_state;
    std::memset(&s, 0, sizeof(FireDev));
    s.dt = dp->dt;
    s.alpha = nag ? dp->momentum : 0.0;
    s.mu = nag ? dp->momentum : 0.0;
    s.method = dp->method;
    s.c_v = 1.0;
    s.c_F = 0.0;
    s.step = resume ? resume->step : 0;
    s.stop_at = s.step;
    s.status = LQ_RUNNING;
    s.init_pending = 1;
    s.tol = dp->force_tol;
    s.max_steps = dp->max_steps;
    return start_controller(lat, s, nag ? v : nullptr);
}

static void fill_report(const FireDev& s, lq_fire_report* out) {
    if (!out) return;
    out->step = s.step;
    out->n_pos = s.n_pos;
    out->restarts = s.restarts;
    out->status = s.status;
    out->pad = 0;
    out->dt = s.dt;
    out->alpha = s.alpha;
    out->P = s.P;
    out->normF = std::sqrt(s.nF2);
    out->normv = std::sqrt(s.nv2);
    out->maxF = s.maxF;
}

int lq_fire_step(lq_lattice* lat, int64_t n_steps, lq_fire_report* out) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    if (!lat->bound) return fail(lat, LQ_ESTATE, "no minimizer is bound to this lattice");
    if (n_steps < 0) return fail(lat, LQ_EINVAL, "n_steps < 0");
    HIPCHK(lat, hipSetDevice(lat->device));
    const void* bufs = lat->p.prec == LQ_F64 ? (const void*)&lat->b64 : (const void*)&lat->b32;
    int rc = launch_begin(lat->d_state, n_steps, lat->stream);
    if (rc == LQ_OK) rc = launch_fire_steps(lat->dev, lat->l23, lat->p.prec, lat->method, bufs, lat->d_partials,
                                            lat->d_state, n_steps, lat->stream);
    if (rc == LQ_OK)
        rc = launch_finalize(lat->dev, lat->p.prec, lat->method != LQ_METHOD_GD, bufs, lat->d_state, lat->stream);
    if (rc != LQ_OK) return fail(lat, rc, "kernel launch failed");
    HIPCHK(lat, hipMemcpyAsync(lat->h_state, lat->d_state, sizeof(FireDev), hipMemcpyDeviceToHost, lat->stream));
    HIPCHK(lat, hipStreamSynchronize(lat->stream));
    fill_report(*lat->h_state, out);
    if (lat->h_state->status == LQ_NONFINITE) return fail(lat, LQ_ENONFINITE, "a step reduction is not finite");
    return LQ_OK;
}

// Steps the bound minimizer until it stops (chunks of growing length, so a
// run that converges early is not stepped far past its stop), then
// evaluates the energy of the final state.
static int run_to_stop(lq_lattice* lat, int64_t max_steps, lq_min_result* out) {
    lq_fire_report r{};
    fill_report(*lat->h_state, &r);
    int rc = LQ_OK;
    int64_t chunk = 64;
    while (r.status == LQ_RUNNING) {
        rc = lq_fire_step(lat, std::min<int64_t>(chunk, max_steps - r.step), &r);
        if (rc != LQ_OK) break;
        chunk = std::min<int64_t>(chunk * 2, 1024);
    }
    lq_energy_terms e{};
    e.bulk = e.elastic = e.anchoring = e.external = e.total = NAN;
    e.n_sim = lat->n_sim;
    if (rc == LQ_OK) rc = lq_energy(lat, lat->q, &e);
    if (out) {
        out->fire = r;
        out->energy = e;
        out->normF_per_site = lat->n_sim > 0 ? r.normF / std::sqrt((double)lat->n_sim) : 0.0;
    }
    return rc;
}

int lq_minimize(lq_lattice* lat, const lq_fire_params* fp, void* q, void* v, void* F, void* workspace,
                int64_t workspace_bytes, lq_min_result* out) {
    int rc = lq_fire_init(lat, fp, q, v, F, workspace, workspace_bytes, nullptr);
    if (rc != LQ_OK) return rc;
    return run_to_stop(lat, fp->max_steps, out);
}

int lq_descent_minimize(lq_lattice* lat, const lq_descent_params* dp, void* q, void* v, void* F, void* workspace,
                        int64_t workspace_bytes, lq_min_result* out) {
    int rc = lq_descent_init(lat, dp, q, v, F, workspace, workspace_bytes, nullptr);
    if (rc != LQ_OK) return rc;
    return run_to_stop(lat, dp->max_steps, out);
}

int lq_minimize_noalloc(lq_lattice* lat, const lq_fire_params* fp, void* q, void* v, void* F,
                        lq_min_result* out) {
    if (!lat) return fail(nullptr, LQ_EINVAL, "lattice is NULL");
    lat->bound = false;
    const int64_t need = lq_workspace_bytes(lat);
    if (need > LQ_NOALLOC_WORKSPACE_BYTES) {
        char msg[192];
        std::snprintf(msg, sizeof msg,
                      "lattice needs %lld bytes of FIRE workspace; lq_minimize_noalloc holds at most %lld "
                      "(use lq_minimize with a caller-allocated workspace)",
                      (long long)need, (long long)LQ_NOALLOC_WORKSPACE_BYTES);
        return fail(lat, LQ_ENOMEM, msg);
    }
    HIPCHK(lat, hipSetDevice(lat->device));
    void* ws = nullptr;
    int rc = noalloc_workspace(lat->device, &ws);
    if (rc != LQ_OK) return fail(lat, rc, "device address of the fixed workspace not available");
    rc = lq_fire_init(lat, fp, q, v, F, ws, LQ_NOALLOC_WORKSPACE_BYTES, nullptr);
    if (rc == LQ_OK) rc = run_to_stop(lat, fp->max_steps, out);
    // the next call on this GPU may reuse the array: nothing may continue from it
    lat->bound = false;
    return rc;
}

int lq_stream_copy(const void* const* src, void* const* dst, int32_t n_streams, int64_t bytes, int32_t width,
                   void* stream) {
    if (!src || !dst || n_streams < 1 || n_streams > STREAMS_MAX)
        return fail(nullptr, LQ_EINVAL, "n_streams must lie in 1..16 with src and dst arrays");
    if (width != 4 && width != 8 && width != 16) return fail(nullptr, LQ_EINVAL, "width must be 4, 8 or 16 bytes");
    if (bytes <= 0 || bytes > ((int64_t)1 << 31) || bytes % width != 0)
        return fail(nullptr, LQ_EINVAL, "bytes must be a positive multiple of width, at most 2^31");
    StreamSet p{};
    for (int i = 0; i < n_streams; ++i) {
        if (!src[i] || !dst[i] || ((uintptr_t)src[i] % 16) != 0 || ((uintptr_t)dst[i] % 16) != 0)
            return fail(nullptr, LQ_EINVAL, "stream buffers must be non-NULL and 16-byte aligned");
        p.src[i] = src[i];
        p.dst[i] = dst[i];
    }
    const int rc = launch_stream_copy(p, n_streams, bytes, width, stream);
    if (rc != LQ_OK) return fail(nullptr, rc, "kernel launch failed");
    return LQ_OK;
}

const char* lq_last_error(const lq_lattice* lat) { return lat ? lat->err.c_str() : g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// batches
struct lq_batch {
    int capacity = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<lq_lattice*> members;
    int prec = -1;
    bool l23 = false;
    MemberDev* d_mem = nullptr;
    int* d_tile_off = nullptr;   // narrow group's offsets, then the wide group's
    int* d_fin_off = nullptr;
    FireDev* d_gather = nullptr;
    MemberDev* h_mem = nullptr;  // pinned, device order: narrow-tile members first
    int* h_off = nullptr;        // pinned: tile offsets (capacity + 2), then finalize offsets (capacity + 1)
    FireDev* h_gather = nullptr; // pinned, device order
    std::vector<int> order;      // device order -> index in members
};

// Removes a lattice that is being destroyed from its batch, after the
// batch's queued work has finished.
static void leave_batch(lq_lattice* lat) {
    lq_batch* b = lat->batch;
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    for (size_t i = 0; i < b->members.size(); ++i)
        if (b->members[i] == lat) {
            b->members.erase(b->members.begin() + (long)i);
            break;
        }
    lat->batch = nullptr;
}

static int fin_blocks_of(const lq_lattice* lat) {
    const int64_t n = 5 * lat->N;
    const int64_t b = (n + 256 * 8 - 1) / (256 * 8);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

extern "C" {

int lq_batch_create(int32_t capacity, void* stream, lq_batch** out) {
    if (!out) return fail(nullptr, LQ_EINVAL, "out is NULL");
    *out = nullptr;
    if (capacity < 1 || capacity > 65536) return fail(nullptr, LQ_EINVAL, "capacity out of range");
    lq_batch* b = new lq_batch();
    b->capacity = capacity;
    b->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipMalloc(&b->d_mem, sizeof(MemberDev) * capacity);
    if (e == hipSuccess) e = hipMalloc(&b->d_tile_off, sizeof(int) * (capacity + 2));
    if (e == hipSuccess) e = hipMalloc(&b->d_fin_off, sizeof(int) * (capacity + 1));
    if (e == hipSuccess) e = hipMalloc(&b->d_gather, sizeof(FireDev) * capacity);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_mem, sizeof(MemberDev) * capacity, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_off, sizeof(int) * (2 * capacity + 3), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_gather, sizeof(FireDev) * capacity, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        lq_batch_destroy(b);
        return fail(nullptr, LQ_ENOMEM, std::string("batch allocation failed: ") + hipGetErrorString(e));
    }
    *out = b;
    return LQ_OK;
}

int lq_batch_destroy(lq_batch* b) {
    if (!b) return LQ_OK;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    for (lq_lattice* m : b->members) m->batch = nullptr;
    if (b->d_mem) (void)hipFree(b->d_mem);
    if (b->d_tile_off) (void)hipFree(b->d_tile_off);
    if (b->d_fin_off) (void)hipFree(b->d_fin_off);
    if (b->d_gather) (void)hipFree(b->d_gather);
    if (b->h_mem) (void)hipHostFree(b->h_mem);
    if (b->h_off) (void)hipHostFree(b->h_off);
    if (b->h_gather) (void)hipHostFree(b->h_gather);
    delete b;
    return LQ_OK;
}

int32_t lq_batch_size(const lq_batch* b) { return b ? (int32_t)b->members.size() : 0; }

int lq_batch_add(lq_batch* b, lq_lattice* lat) {
    if (!b || !lat) return fail(lat, LQ_EINVAL, "batch or lattice is NULL");
    if (!lat->bound) return fail(lat, LQ_ESTATE, "lattice is not bound by lq_fire_init");
    if (lat->method != LQ_METHOD_FIRE) return fail(lat, LQ_EINVAL, "batched stepping runs FIRE only");
    if ((int)b->members.size() >= b->capacity) return fail(lat, LQ_EINVAL, "batch is full");
    if (lat->device != b->device) return fail(lat, LQ_EINVAL, "lattice and batch are on different devices");
    if (lat->batch == b) return fail(lat, LQ_EINVAL, "lattice is a member already");
    if (lat->batch) return fail(lat, LQ_EINVAL, "lattice is a member of another batch");
    if (!b->members.empty() && (lat->p.prec != b->prec || lat->l23 != b->l23))
        return fail(lat, LQ_EINVAL, "members must share prec and the use of L2/L3");
    HIPCHK(lat, hipSetDevice(lat->device));
    HIPCHK(lat, hipStreamSynchronize(lat->stream));
    if (b->members.empty()) {
        b->prec = lat->p.prec;
        b->l23 = lat->l23;
    }
    b->members.push_back(lat);
    lat->batch = b;
    return LQ_OK;
}

int lq_batch_remove(lq_batch* b, lq_lattice* lat) {
    if (!b || !lat) return fail(lat, LQ_EINVAL, "batch or lattice is NULL");
    for (size_t i = 0; i < b->members.size(); ++i)
        if (b->members[i] == lat) {
            b->members.erase(b->members.begin() + (long)i);
            lat->batch = nullptr;
            return LQ_OK;
        }
    return fail(lat, LQ_EINVAL, "lattice is not a member");
}

int lq_batch_step(lq_batch* b, int64_t n_steps, lq_fire_report* reports) {
    if (!b) return fail(nullptr, LQ_EINVAL, "batch is NULL");
    if (n_steps < 0) return fail(nullptr, LQ_EINVAL, "n_steps < 0");
    const int n = (int)b->members.size();
    if (n == 0) return LQ_OK;
    if (!reports) return fail(nullptr, LQ_EINVAL, "reports is NULL");
    HIPCHK(nullptr, hipSetDevice(b->device));
    for (lq_lattice* m : b->members)
        if (!m->bound) return fail(nullptr, LQ_ESTATE, "a member lost its FIRE binding; remove it or bind it again");
    // the descriptors are rebuilt on every call (a few hundred bytes per
    // member), so members re-bound by lq_fire_init are picked up.  Members
    // on narrow tiles come first and run in one launch per step, members on
    // wide tiles in a second one.
    b->order.clear();
    for (int w = 0; w < 2; ++w)
        for (int i = 0; i < n; ++i)
            if (b->members[i]->dev.wide == w) b->order.push_back(i);
    int n_narrow = 0;
    while (n_narrow < n && !b->members[b->order[n_narrow]]->dev.wide) ++n_narrow;
    const int n_wide = n - n_narrow;
    int* tile_off = b->h_off;                     // narrow: [0, n_narrow], wide: [n_narrow + 1, n + 1]
    int* fin_off = b->h_off + (b->capacity + 2);  // [0, n]
    int tiles[2] = {0, 0}, f = 0;
    for (int j = 0; j < n; ++j) {
        lq_lattice* m = b->members[b->order[j]];
        const int grp = j < n_narrow ? 0 : 1;
        MemberDev& d = b->h_mem[j];
        std::memset(&d, 0, sizeof(d));
        d.L = m->dev;
        const Bufs<double>& bb = m->b64;
        for (int k = 0; k < 2; ++k) {
            d.q[k] = bb.q[k];
            d.v[k] = bb.v[k];
            d.F[k] = bb.F[k];
        }
        d.partials = m->d_partials;
        d.st = m->d_state;
        d.nblocks = (int)n_step_blocks(m->dev);
        tile_off[grp == 0 ? j : j + 1] = tiles[grp];
        fin_off[j] = f;
        tiles[grp] += d.nblocks;
        f += fin_blocks_of(m);
    }
    tile_off[n_narrow] = tiles[0];
    tile_off[n + 1] = tiles[1];
    fin_off[n] = f;
    HIPCHK(nullptr, hipMemcpyAsync(b->d_mem, b->h_mem, sizeof(MemberDev) * n, hipMemcpyHostToDevice, b->stream));
    HIPCHK(nullptr, hipMemcpyAsync(b->d_tile_off, tile_off, sizeof(int) * (n + 2), hipMemcpyHostToDevice,
                                   b->stream));
    HIPCHK(nullptr, hipMemcpyAsync(b->d_fin_off, fin_off, sizeof(int) * (n + 1), hipMemcpyHostToDevice, b->stream));
    int rc = launch_batch_steps(b->prec, b->l23, b->d_mem, n_narrow, b->d_tile_off, tiles[0], n_wide,
                                b->d_tile_off + n_narrow + 1, tiles[1], b->d_fin_off, f, b->d_gather, n_steps,
                                b->stream);
    if (rc != LQ_OK) return fail(nullptr, rc, "batch kernel launch failed");
    HIPCHK(nullptr, hipMemcpyAsync(b->h_gather, b->d_gather, sizeof(FireDev) * n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(nullptr, hipStreamSynchronize(b->stream));
    int worst = LQ_OK;
    for (int j = 0; j < n; ++j) {
        const int i = b->order[j];
        fill_report(b->h_gather[j], &reports[i]);
        *b->members[i]->h_state = b->h_gather[j];
        if (b->h_gather[j].status == LQ_NONFINITE) worst = LQ_ENONFINITE;
    }
    if (worst != LQ_OK) return fail(nullptr, worst, "a member's FIRE reduction is not finite");
    return LQ_OK;
}

}  // extern "C"
