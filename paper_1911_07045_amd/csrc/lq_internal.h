// Internal declarations shared by the host side of liblqfire and its kernels.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "lqfire.h"

namespace lq {

// Per-site neighbour mask byte.  Bits 0..5: the face neighbour +x, -x, +y,
// -y, +z, -z exists and is simulated; bit 6: the site itself is simulated;
// bit 7: the site carries anchoring.  Sites inside objects and positions off
// an open edge have mask 0.
constexpr uint8_t M_SIM = 0x40;
constexpr uint8_t M_ANCH = 0x80;
constexpr uint8_t M_FULL = 0x7F;  // simulated bulk site with all six neighbours

// Anchoring form of one site: upper triangle of K (15), b (5), c (1) with
// f = 1/2 q^T K q + b^T q + c.
constexpr int ANCH_STRIDE = 21;
// The force's copy of a row: K upper triangle (15) and b (5), in the field's
// element type.
constexpr int ANCH_FSTRIDE = 20;

// Host-side rasterization result.
struct Geometry {
    std::vector<uint8_t> type;       // 0 bulk, 1 boundary, 2 object
    std::vector<uint8_t> mask;       // neighbour mask (above)
    std::vector<int64_t> anch_site;  // sorted
    std::vector<double> anch_data;   // ANCH_STRIDE per anchored site
    int64_t n_sim = 0;
};

// Returns LQ_OK or an error code with a message in err.
int rasterize(const lq_params& p, double S0, const lq_object* objs, int32_t n_objs,
              const lq_site_anchor* recs, int64_t n_recs, const int64_t* object_sites,
              int64_t n_object_sites, Geometry& g, std::string& err);

// Tile geometry of the fused kernel, per element type, term set and width
// kind: a block of X x Y threads owns an X x Y column tile and marches zc
// planes along z.  Long rows cut the halo's share of the traffic (the two
// x-edge columns of the ring cost one cache line per row for one value
// each), so the wide tile is as wide as the block's register budget allows:
// 1024 threads for the one-constant FP32 kernel (at most 128 VGPRs, four
// waves per SIMD), 512 for FP32 with L2/L3/L4 and for one-constant FP64,
// 256 (64 x 4) for FP64 with L2/L3/L4.  Lattices narrower than a wide tile
// (the small boxes of a serving batch) use a narrow tile instead: 64 x 8 in
// FP32 (on a stream of 16-64-site boxes it gave half the median latency of
// 32 x 8), 32 x 8 in FP64.  WAVES is the number of waves per SIMD a kernel
// is held to (1: no constraint).
#ifndef LQ_TILE_X_F32
#define LQ_TILE_X_F32 128
#endif
#ifndef LQ_TILE_Y_F32
#define LQ_TILE_Y_F32 8
#endif
#ifndef LQ_TILE_X_F32_L23
#define LQ_TILE_X_F32_L23 64
#endif
#ifndef LQ_TILE_Y_F32_L23
#define LQ_TILE_Y_F32_L23 8
#endif
#ifndef LQ_TILE_X_F64
#define LQ_TILE_X_F64 64
#endif
#ifndef LQ_TILE_Y_F64
#define LQ_TILE_Y_F64 8
#endif
#ifndef LQ_TILE_X_F64_L23
#define LQ_TILE_X_F64_L23 64
#endif
#ifndef LQ_TILE_Y_F64_L23
#define LQ_TILE_Y_F64_L23 4
#endif
#ifndef LQ_WAVES_F64_L23
#define LQ_WAVES_F64_L23 1
#endif
template <int TX_, int TY_, int WAVES_>
struct TileGeom {
    static constexpr int X = TX_, Y = TY_;
    static constexpr int N = X * Y;            // threads per block
    static constexpr int PX = X + 2, PY = Y + 2;  // padded tile in LDS
    static constexpr int RING = 2 * PX + 2 * (PY - 2);
    static constexpr int RING_ITEMS = 5 * RING;   // (site, component) pairs of the ring
    static constexpr int IPT = (RING_ITEMS + N - 1) / N;
    static constexpr int WAVES = WAVES_;
};
// W = 1: wide tile, W = 0: narrow tile
template <typename T, bool L23, int W>
struct Tile;
template <>
struct Tile<float, false, 1> : TileGeom<LQ_TILE_X_F32, LQ_TILE_Y_F32, 4> {};
template <>
struct Tile<float, true, 1> : TileGeom<LQ_TILE_X_F32_L23, LQ_TILE_Y_F32_L23, 1> {};
template <>
struct Tile<double, false, 1> : TileGeom<LQ_TILE_X_F64, LQ_TILE_Y_F64, 1> {};
template <>
struct Tile<double, true, 1> : TileGeom<LQ_TILE_X_F64_L23, LQ_TILE_Y_F64_L23, LQ_WAVES_F64_L23> {};
template <bool L23>
struct Tile<float, L23, 0> : TileGeom<64, 8, Tile<float, L23, 1>::WAVES> {};
template <bool L23>
struct Tile<double, L23, 0> : TileGeom<32, 8, Tile<double, L23, 1>::WAVES> {};

template <int W>
inline int tile_x_w(int prec, bool l23) {
    if (prec == LQ_F64) return l23 ? Tile<double, true, W>::X : Tile<double, false, W>::X;
    return l23 ? Tile<float, true, W>::X : Tile<float, false, W>::X;
}
template <int W>
inline int tile_y_w(int prec, bool l23) {
    if (prec == LQ_F64) return l23 ? Tile<double, true, W>::Y : Tile<double, false, W>::Y;
    return l23 ? Tile<float, true, W>::Y : Tile<float, false, W>::Y;
}
inline int tile_x(int prec, bool l23, int wide) { return wide ? tile_x_w<1>(prec, l23) : tile_x_w<0>(prec, l23); }
inline int tile_y(int prec, bool l23, int wide) { return wide ? tile_y_w<1>(prec, l23) : tile_y_w<0>(prec, l23); }
inline int tile_threads(int prec, bool l23, int wide) { return tile_x(prec, l23, wide) * tile_y(prec, l23, wide); }
// a lattice narrower than one wide tile takes the narrow one
inline int tile_wide_for(int64_t nx, int prec, bool l23) { return nx >= tile_x_w<1>(prec, l23) ? 1 : 0; }

// One block's work in the step kernels: the X x Y column tile at (x0, y0)
// over planes z0 .. z0 + zc - 1, zc <= CHUNK_MAX.
struct Chunk {
    int32_t x0, y0, z0, zc;
};
// Per-chunk plane flags: bit i % 64 of word i / 64 is set when plane z0 + i
// and both its z-neighbours are M_FULL over the padded tile.
constexpr int PLANE_WORDS = 4;
constexpr int CHUNK_MAX = 64 * PLANE_WORDS;
struct PlaneBits {
    uint64_t w[PLANE_WORDS];
};

// Device view of a lattice.
struct LatDev {
    int nx, ny, nz;
    int per[3];
    int64_t N;
    const uint8_t* mask;
    const Chunk* chunks;       // of the step kernels, in block order
    const int32_t* first;      // block b of the step kernels marches chunks first[b] .. first[b + 1] - 1
    const uint8_t* tile_bulk;  // per chunk, 1: every site of the padded tile has mask M_FULL
    const PlaneBits* tile_planes;  // per chunk
    int n_anch;
    const int32_t* anch_index;  // per site: 1 + row of anch_data, 0 when not anchored
    const double* anch_data;    // ANCH_STRIDE per anchored site
    const void* anch_force;     // ANCH_FSTRIDE per anchored site, element type of the field
    double ext[5];              // constant external-field force per simulated site
    double A, B, C, L1, L2, L3, L4;
    int nchunks;  // chunks of one step launch
    int nblocks;  // blocks of one step launch
    int wide;     // tile width kind of the step kernels (1 wide, 0 narrow)
    int two_waves;  // FP64 L2/L3 wide: the step kernels held to two waves per SIMD
};

// FIRE state kept in device memory.
struct FireDev {
    double dt, alpha;
    double c_v, c_F;  // steering still to be applied to the stored v
    int64_t n_pos, step, restarts, stop_at;
    int32_t cur;      // which of the two buffers holds the current state
    int32_t done;     // no further step in this call
    int32_t status;   // LQ_RUNNING / LQ_CONVERGED / LQ_MAX_STEPS / LQ_NONFINITE
    int32_t init_pending;  // the next reduction is the one of lq_fire_init
    double P, nF2, nv2, maxF;
    double dt_max, alpha0, f_inc, f_dec, f_alpha, tol;
    int64_t n_min, max_steps;
    uint32_t ticket;
    int32_t method;   // LQ_METHOD_FIRE / LQ_METHOD_GD / LQ_METHOD_NESTEROV
    double mu;        // Nesterov momentum
};

// The state of a lattice's step kernels: FireDev st[2] followed by DcCtl.
// st[0] holds the controller state between calls.  Within a call, step
// kernel k (1-based) first runs the controller on the reduction of step
// k - 1 (every block, identically) and block 0 stores the result in
// st[(k - 1) & 1]; a block that finds the run stopped sets halt.
struct DcCtl {
    int32_t halt;  // a step kernel of this call found the run stopped
    int32_t slot;  // ... and left the final state in st[slot]
};

// march kernel variants
enum : int { MODE_FORCE = 0, MODE_FIRE = 1, MODE_GD = 2, MODE_NAG = 3 };

template <typename T>
struct Bufs {
    T* q[2];
    T* v[2];
    T* F[2];
};

// One member of a batch (device copy).
struct MemberDev {
    LatDev L;
    void* q[2];
    void* v[2];
    void* F[2];
    double* partials;
    FireDev* st;
    int nblocks;  // step tiles of this member
    int pad;
};

struct EnergyOut {
    double bulk, elastic, anch, ext;
};

// Kernel launchers (kernels.hip).  All enqueue on stream.
int launch_forces(const LatDev& L, bool l23, int prec, const void* q, void* F, void* stream);
int launch_fire_init_reduce(const LatDev& L, int prec, const void* F, const void* v,
                            double* partials, FireDev* st, void* stream);
int launch_fire_steps(const LatDev& L, bool l23, int prec, int method, const void* bufs, double* partials,
                      FireDev* st, int64_t n_steps, void* stream);
int launch_begin(FireDev* st, int64_t n_steps, void* stream);
int launch_finalize(const LatDev& L, int prec, bool with_v, const void* bufs, FireDev* st, void* stream);
int launch_lookahead(const LatDev& L, int prec, const void* q, const void* m, double mu, void* y,
                     void* stream);
int launch_fill_zero(void* p, int64_t bytes, void* stream);
int launch_directors(const LatDev& L, int prec, const void* q, void* dirs, void* lmax, uint8_t* defect,
                     double thr, unsigned long long* count, void* stream);
int launch_energy(const LatDev& L, bool l23, int prec, const void* q, double* partials,
                  EnergyOut* out, uint32_t* ticket, void* stream);
int launch_uniaxial(const LatDev& L, int prec, const double* dirs, double S, void* q,
                    void* stream);
// Members [0, n_narrow) of mem use narrow tiles, the next n_wide wide ones;
// tile_off / tile_off_wide hold each group's cumulative tile offsets.
int launch_batch_steps(int prec, bool l23, const MemberDev* mem, int n_narrow, const int* tile_off,
                       int tiles_narrow, int n_wide, const int* tile_off_wide, int tiles_wide,
                       const int* fin_off, int total_fin, FireDev* gather, int64_t n_steps, void* stream);
int64_t n_step_blocks(const LatDev& L);
int step_blocks_per_cu(int prec, bool l23, bool l4, int wide, bool two);
int64_t n_energy_blocks(const LatDev& L);

}  // namespace lq
