// HIP kernels of liblqfire for gfx950: the discrete Landau-de Gennes force,
// the fused force + FIRE step, the FIRE controller, the energy and helpers.
//
// The energy is the paper's discretization (sec. III.B): bulk Eq. (fphase),
// distortion Eq. (fdistortionFull) (L6 = 0) from one-sided differences
// Eq. (onesidedderivatives) averaged over every allowed forward/backward
// choice per axis, plus anchoring (sec. II.A.4) and external fields
// (sec. II.A.3).  Because the choices on different axes are independent, the
// average factorizes:
//   - products of differences along one axis k average to the mean over the
//     allowed choices of that axis, which turns the L1 term and the same-axis
//     part of L2/L3 into bond sums, bond (x, x+e_k) weighted
//     w = 1/n_k(x) + 1/n_k(x+e_k) with n_k the number of allowed choices;
//   - products of differences along two different axes j != k average to
//     C_j C_k, with C_k the mean of the allowed one-sided differences of
//     axis k (a central difference in the bulk).
// The forces are the exact negative gradient of that energy with respect to
// the five components q (sec. III.B), i.e. P^T applied to dE/dQ where
// P^T G = (Gxx - Gzz, Gxy + Gyx, Gxz + Gzx, Gyy - Gzz, Gyz + Gzy).
//
// FIRE (Algorithm 1) is fused with the force: the kernel of step t reads
// q, v, F of step t-1 with the steering coefficients (c_v, c_F) and dt
// decided by the controller of step t-1, applies steering, the first half
// kick and the drift to every site it needs (its tile plus a one-site halo,
// recomputed in LDS), evaluates the force at the new positions, applies the
// second half kick and writes q, v, F to the other buffer.  Per-block FP64
// partial sums of F.v, |F|^2, |v|^2 and max|F_i| are combined by the last
// block to finish (atomic ticket), which then runs the controller.  The host
// never waits between steps.  The same march runs gradient descent and
// Nesterov's accelerated gradient (a compile-time mode) and the force alone.
// Further kernels: the energy (FP64 per-term sums), the uniaxial initial
// state, the FIRE bookkeeping, batched steps over many lattices, and the
// director / defect extraction.
//
// Layout: SoA fields [5][nz][ny][nx].  A block owns an X x Y column tile and
// marches zc planes along z, keeping the drifted q of four planes with their
// halo in LDS: the force of plane f reads planes f-1, f, f+1 while plane f+1
// is being written, so that one barrier per plane suffices.
#include <hip/hip_runtime.h>

#include "lq_internal.h"

namespace lq {


__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }

// Raw buffer access to one field (5 components, 5 N elements): the resource
// covers exactly the field, so an offset past its end reads 0 and drops the
// store; the component offset c N sizeof(T) goes in the scalar offset and the
// site offset in one 32-bit vector register.  A field must fit in 2^32 bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    }
}
// Stores of the streamed fields: POL is the buffer instruction's
// cache-policy operand, 2 (bit 1) the non-temporal policy on gfx950, 0 the
// default one.
template <typename T, int POL>
__device__ __forceinline__ void bst_p(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T v) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, POL);
    } else {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, POL);
    }
}
// Cache policy of a step kernel's state stores.  Non-temporal stores keep
// the written state from displacing lines the step still reuses: measured
// faster for the one-constant and the FP64 kernels (5% on the 256^3 boxes).
// The FP32 L2/L3 kernels measured faster with the default policy at every
// size (14% on the 128^3 bulk box, whose two state buffers fit in the
// 256 MiB Infinity Cache, 2-4% on the 512^3 patterned wall).  A compile-time
// choice: a run-time one put a branch in the march loop that cost 1.5%.
template <typename T, bool L23>
constexpr int store_policy() { return (L23 && sizeof(T) == 4) ? 0 : 2; }

// Barrier for data exchanged through LDS only: waits for this wave's LDS
// operations, not for its global loads and stores (which __syncthreads()
// would drain, stalling every plane on memory latency).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ int wrapc(int g, int n, int per) {
    if (g >= 0 && g < n) return g;
    if (!per) return -1;
    g %= n;
    return g < 0 ? g + n : g;
}

__device__ __forceinline__ bool has_nb(uint32_t m, int k, int s) {
    return (m >> (2 * k + (s < 0 ? 1 : 0))) & 1u;
}

__device__ __forceinline__ int n_choices(uint32_t m, int k) {
    return (int)((m >> (2 * k)) & 1u) + (int)((m >> (2 * k + 1)) & 1u);
}

// Coefficients of C_k(x) = ap Q(x+e_k) + a0 Q(x) + am Q(x-e_k): the mean of
// the allowed one-sided differences along axis k.
template <typename T>
__device__ __forceinline__ void mean_diff_coef(uint32_t m, int k, T& ap, T& a0, T& am) {
    bool p = has_nb(m, k, +1), n = has_nb(m, k, -1);
    if (p && n) {
        ap = T(0.5); a0 = T(0); am = T(-0.5);
    } else if (p) {
        ap = T(1); a0 = T(-1); am = T(0);
    } else if (n) {
        ap = T(0); a0 = T(1); am = T(-1);
    } else {
        ap = T(0); a0 = T(0); am = T(0);
    }
}

template <typename T>
__device__ __forceinline__ void full_of(const T q[5], T Q[3][3]) {
    Q[0][0] = q[0]; Q[0][1] = q[1]; Q[0][2] = q[2];
    Q[1][0] = q[1]; Q[1][1] = q[3]; Q[1][2] = q[4];
    Q[2][0] = q[2]; Q[2][1] = q[4]; Q[2][2] = -q[0] - q[3];
}

template <typename T>
__device__ __forceinline__ void pT(const T G[3][3], T g[5]) {
    g[0] = G[0][0] - G[2][2];
    g[1] = G[0][1] + G[1][0];
    g[2] = G[0][2] + G[2][0];
    g[3] = G[1][1] - G[2][2];
    g[4] = G[1][2] + G[2][1];
}

// d(bulk)/dq = P^T (A Q + B Q^2 + C tr(Q^2) Q), written out in the five
// components: P^T Q = M q and P^T S = (Sxx - Szz, 2 Sxy, 2 Sxz, Syy - Szz,
// 2 Syz) for the symmetric S = Q^2.
template <typename T>
__device__ __forceinline__ void bulk_grad(const T q[5], T A, T B, T C, T g[5]) {
    const T zz = -q[0] - q[3];
    const T s01 = q[1] * q[1], s02 = q[2] * q[2], s04 = q[4] * q[4];
    const T t2 = q[0] * q[0] + q[3] * q[3] + zz * zz + T(2) * (s01 + s02 + s04);
    const T Sxx = q[0] * q[0] + s01 + s02;
    const T Syy = s01 + q[3] * q[3] + s04;
    const T Szz = s02 + s04 + zz * zz;
    const T Sxy = q[0] * q[1] + q[1] * q[3] + q[2] * q[4];
    const T Sxz = q[0] * q[2] + q[1] * q[4] + q[2] * zz;
    const T Syz = q[1] * q[2] + q[3] * q[4] + q[4] * zz;
    const T a = A + C * t2;
    g[0] = a * (T(2) * q[0] + q[3]) + B * (Sxx - Szz);
    g[1] = T(2) * (a * q[1] + B * Sxy);
    g[2] = T(2) * (a * q[2] + B * Sxz);
    g[3] = a * (q[0] + T(2) * q[3]) + B * (Syy - Szz);
    g[4] = T(2) * (a * q[4] + B * Syz);
}

// The bond (L1) metric: sum_ij dQ_ij^2 = d^T M d; returns M d.
template <typename T>
__device__ __forceinline__ void metric(const T d[5], T o[5]) {
    o[0] = T(2) * d[0] + d[3];
    o[1] = T(2) * d[1];
    o[2] = T(2) * d[2];
    o[3] = d[0] + T(2) * d[3];
    o[4] = T(2) * d[4];
}

// Same-axis part of L2/L3 along axis j: sum_i dQ_ij^2 (column j of dQ);
// returns its gradient / 2 with respect to d.
template <typename T>
__device__ __forceinline__ void column_metric(int j, const T d[5], T o[5]) {
    if (j == 0) {
        o[0] = d[0]; o[1] = d[1]; o[2] = d[2]; o[3] = T(0); o[4] = T(0);
    } else if (j == 1) {
        o[0] = T(0); o[1] = d[1]; o[2] = T(0); o[3] = d[3]; o[4] = d[4];
    } else {
        T s = d[0] + d[3];
        o[0] = s; o[1] = T(0); o[2] = d[2]; o[3] = s; o[4] = d[4];
    }
}

// h_j = P^T H_j with H_j,ab = sum_{k != j} [L2 delta_bj C_k,ak + L3 delta_bk C_k,aj]:
// the derivative of the cross-axis L2/L3 energy of one site with respect to
// its mean difference C_j, mapped to q components.
template <typename T>
__device__ __forceinline__ void cross_h(int j, const T Ck[3][5], T L2, T L3, T h[5]) {
    T H[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) H[a][b] = T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k == j) continue;
        T C[3][3];
        full_of(Ck[k], C);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            H[a][j] += L2 * C[a][k];
            H[a][k] += L3 * C[a][j];
        }
    }
    pT(H, h);
}

// Levi-Civita symbol
__host__ __device__ constexpr int eps3(int a, int b, int c) { return ((a - b) * (b - c) * (c - a)) / 2; }

// Chiral term (L4) of Eq. (fdistortionFull), E4(x) = L4/2 eps_lik Q_lj(x) C_k,ij(x).
// Its derivative with respect to the site tensor: P^T of sum_ik eps_aik C_k,ib.
template <typename T>
__device__ __forceinline__ void chiral_site(const T C[3][5], T h[5]) {
    T H[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) H[a][b] = T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T Ck[3][3];
        full_of(C[k], Ck);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (eps3(a, i, k) == 0) continue;
#pragma unroll
                for (int b = 0; b < 3; ++b) H[a][b] += T(eps3(a, i, k)) * Ck[i][b];
            }
    }
    pT(H, h);
}

// Derivative of E4(x) with respect to the tensor of a site that enters C_k(x)
// with coefficient 1: P^T of sum_l eps_lak Q_lb(x).
template <typename T>
__device__ __forceinline__ void chiral_nb(int k, const T qx[5], T h[5]) {
    T Qx[3][3], H[3][3];
    full_of(qx, Qx);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            T v = T(0);
#pragma unroll
            for (int l = 0; l < 3; ++l)
                if (eps3(l, a, k) != 0) v += T(eps3(l, a, k)) * Qx[l][b];
            H[a][b] = v;
        }
    pT(H, h);
}

// ---------------------------------------------------------------------------
// Stencil view used by the force: offsets (dx, dy, dz) in {-1, 0, 1} around
// the centre, read from the LDS slots of the planes below, at and above the
// centre.  BULK: every site of the padded tile is simulated with all six
// neighbours, so masks are compile-time constants.
template <typename T, bool L23, bool BULK, int W>
struct Stencil {
    T (*q)[5][Tile<T, L23, W>::PY][Tile<T, L23, W>::PX];
    uint8_t (*m)[Tile<T, L23, W>::PY][Tile<T, L23, W>::PX];
    int s[3];  // LDS slots of the planes below, at and above the centre
    int cx, cy;
    __device__ __forceinline__ T at(int dx, int dy, int dz, int c) const {
        return q[s[dz + 1]][c][cy + dy][cx + dx];
    }
    __device__ __forceinline__ uint32_t mask(int dx, int dy, int dz) const {
        if (BULK) return (uint32_t)M_FULL;
        return (uint32_t)m[s[dz + 1]][cy + dy][cx + dx];
    }
    __device__ __forceinline__ void load5(int dx, int dy, int dz, T o[5]) const {
#pragma unroll
        for (int c = 0; c < 5; ++c) o[c] = at(dx, dy, dz, c);
    }
};

__device__ __forceinline__ void unit(int k, int s, int& dx, int& dy, int& dz) {
    dx = k == 0 ? s : 0;
    dy = k == 1 ? s : 0;
    dz = k == 2 ? s : 0;
}

// The FP32 L2/L3 kernels evaluate boundary sites branch-free: every stencil
// position holds a finite value (0 where no simulated site is), so a term
// whose coefficient is 0 adds exactly nothing, and the LDS reads of all
// terms can be in flight together (the branch per term serialized them on
// LDS latency; measured 33% faster on the 128^3 colloid slab).  In FP64 the
// branch-free form needs more registers than the kernel has and measured
// slower, so the FP64 kernels read only the terms that are present.
template <typename T>
constexpr bool branch_free() { return sizeof(T) == 4; }

// mean differences C_k (k != skip) at offset o of the stencil
template <typename T, bool L23, bool BULK, int W>
__device__ __forceinline__ void mean_diffs(const Stencil<T, L23, BULK, W>& P, int ox, int oy, int oz,
                                           int skip, uint32_t m, T Ck[3][5]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k == skip) {
#pragma unroll
            for (int c = 0; c < 5; ++c) Ck[k][c] = T(0);
            continue;
        }
        T ap, a0, am;
        mean_diff_coef(m, k, ap, a0, am);
        int ex, ey, ez;
        unit(k, 1, ex, ey, ez);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            T v = a0 * P.at(ox, oy, oz, c);
            if (branch_free<T>() || ap != T(0)) v = fma_t(ap, P.at(ox + ex, oy + ey, oz + ez, c), v);
            if (branch_free<T>() || am != T(0)) v = fma_t(am, P.at(ox - ex, oy - ey, oz - ez, c), v);
            Ck[k][c] = v;
        }
    }
}

// K (upper triangle) and b of one site's anchoring form
template <typename T>
struct AnchRow {
    T k[15], b[5];
};

// Loads the force's copy of anchoring row arow1 - 1 (zeros for arow1 == 0:
// the offset lies past the end of the buffer).
template <typename T>
__device__ __forceinline__ void anch_load(const LatDev& L, int arow1, AnchRow<T>& A) {
    constexpr uint32_t ROW = ANCH_FSTRIDE * sizeof(T);  // 80 or 160 bytes: whole 16-byte pieces
    const __amdgpu_buffer_rsrc_t r = field_rsrc(L.anch_force, (uint32_t)L.n_anch * ROW);
    const uint32_t off = arow1 > 0 ? (uint32_t)(arow1 - 1) * ROW : 0xFFFFFFFFu;
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    T v[ANCH_FSTRIDE];
#pragma unroll
    for (int i = 0; i < (int)(ROW / 16); ++i) {
        // whole-vector casts: a bit cast of one subscripted element of the
        // loaded vector is not reliably compiled
        const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, i * 16, 0);
        if constexpr (sizeof(T) == 4) {
            const f32x4 x = __builtin_bit_cast(f32x4, w);
            v[4 * i + 0] = x.x; v[4 * i + 1] = x.y; v[4 * i + 2] = x.z; v[4 * i + 3] = x.w;
        } else {
            const f64x2 x = __builtin_bit_cast(f64x2, w);
            v[2 * i + 0] = x.x; v[2 * i + 1] = x.y;
        }
    }
#pragma unroll
    for (int i = 0; i < 15; ++i) A.k[i] = v[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) A.b[i] = v[15 + i];
}

// -dE/dq at the stencil centre (a simulated site with mask m0).  Where m0
// carries the anchoring bit, the site's anchoring form is AR (wide tiles,
// loaded ahead by the caller) or row arow1 - 1 of the FP64 forms, read here
// (narrow tiles: on the serving stream of small boxes this measured a lower
// tail latency than the early loads; FP64 L2/L3: the 40 registers of an early
// row are what keeps that kernel from two waves per SIMD).
template <typename T, bool L23, bool L4, bool BULK, int W>
__device__ __forceinline__ void site_force(const Stencil<T, L23, BULK, W>& P, uint32_t m0,
                                           const LatDev& L, const AnchRow<T>& AR, int arow1, T F[5]) {
    const T A = T(L.A), B = T(L.B), C = T(L.C), L1 = T(L.L1);
    T q0[5];
    P.load5(0, 0, 0, q0);
    T g[5];
    bulk_grad(q0, A, B, C, g);
    // external fields: a constant force per simulated site
#pragma unroll
    for (int c = 0; c < 5; ++c) g[c] -= T(L.ext[c]);
    if (BULK) {
        // every bond has weight 1: the L1 term is -L1 M (sum of neighbours - 6 q)
        T S[3][5];  // q(+e_k) + q(-e_k)
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            S[0][c] = P.at(1, 0, 0, c) + P.at(-1, 0, 0, c);
            S[1][c] = P.at(0, 1, 0, c) + P.at(0, -1, 0, c);
            S[2][c] = P.at(0, 0, 1, c) + P.at(0, 0, -1, c);
            F[c] = fma_t(T(-6), q0[c], (S[0][c] + S[1][c]) + S[2][c]);
        }
        T o[5];
        metric(F, o);
#pragma unroll
        for (int c = 0; c < 5; ++c) g[c] = fma_t(-L1, o[c], g[c]);
        if (L23) {
            // In the bulk every mean difference is central and both L2/L3
            // parts depend on L2 + L3 only.  Same-axis part: (L2 + L3) times
            // the sum over axes k of column k of (2 q - S_k).  Cross-axis
            // part: the sum over x = centre -+ e_j of +-1/2 h_j(x) collapses
            // to -1/4 (L2 + L3) sum_{j<k} X_jk, where X_jk = P^T H with
            // H_aj = D_ak, H_ak = D_aj, and D the full tensor of the mixed
            // second difference q(+j+k) - q(+j-k) - q(-j+k) + q(-j-k).
            // Written out, X_xy = (D1, D0 + D3, D4, D1, D2),
            // X_xz = (0, D4, -D3, -D2, D1), X_yz = (-D4, D2, D1, 0, -D0).
            T d[3][5];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int c = 0; c < 5; ++c) d[k][c] = fma_t(T(2), q0[c], -S[k][c]);
            const T s2 = d[2][0] + d[2][3];
            T col[5];
            col[0] = d[0][0] + s2;
            col[1] = d[0][1] + d[1][1];
            col[2] = d[0][2] + d[2][2];
            col[3] = d[1][3] + s2;
            col[4] = d[1][4] + d[2][4];
            auto mix = [&](int j, int k, int c) {
                int pj[3], pk[3];
                unit(j, 1, pj[0], pj[1], pj[2]);
                unit(k, 1, pk[0], pk[1], pk[2]);
                return (P.at(pj[0] + pk[0], pj[1] + pk[1], pj[2] + pk[2], c) -
                        P.at(pj[0] - pk[0], pj[1] - pk[1], pj[2] - pk[2], c)) -
                       (P.at(pk[0] - pj[0], pk[1] - pj[1], pk[2] - pj[2], c) -
                        P.at(-pj[0] - pk[0], -pj[1] - pk[1], -pj[2] - pk[2], c));
            };
            T X[5];
            X[0] = mix(0, 1, 1) - mix(1, 2, 4);
            X[1] = (mix(0, 1, 0) + mix(0, 1, 3)) + (mix(0, 2, 4) + mix(1, 2, 2));
            X[2] = (mix(0, 1, 4) - mix(0, 2, 3)) + mix(1, 2, 1);
            X[3] = mix(0, 1, 1) - mix(0, 2, 2);
            X[4] = (mix(0, 1, 2) + mix(0, 2, 1)) - mix(1, 2, 0);
            const T L23s = T(L.L2) + T(L.L3);
#pragma unroll
            for (int c = 0; c < 5; ++c) g[c] = fma_t(L23s, fma_t(T(-0.25), X[c], col[c]), g[c]);
        }
    } else {
        // bond sums: L1 and the same-axis part of L2/L3.  Branch-free (FP32
        // L2/L3): an absent bond gets weight 0; the other kernels skip it.
        constexpr bool BF = L23 && branch_free<T>();
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int s = -1; s <= 1; s += 2) {
                if (!BF && !has_nb(m0, k, s)) continue;
                int dx, dy, dz;
                unit(k, s, dx, dy, dz);
                uint32_t mn = P.mask(dx, dy, dz);
                T w = (n_choices(m0, k) == 2 ? T(0.5) : T(1)) + (n_choices(mn, k) == 2 ? T(0.5) : T(1));
                w = has_nb(m0, k, s) ? w : T(0);
                T d[5], o[5];
#pragma unroll
                for (int c = 0; c < 5; ++c) d[c] = q0[c] - P.at(dx, dy, dz, c);
                metric(d, o);
                T wl = w * L1;
#pragma unroll
                for (int c = 0; c < 5; ++c) g[c] = fma_t(wl, o[c], g[c]);
                if (L23) {
                    column_metric(k, d, o);
                    T wl23 = w * (T(L.L2) + T(L.L3));
#pragma unroll
                    for (int c = 0; c < 5; ++c) g[c] = fma_t(wl23, o[c], g[c]);
                }
                // one bond's reads at a time in flight: hoisting every
                // stencil read of the branch-free form spills registers
                if (BF) __builtin_amdgcn_sched_barrier(0);
            }
    }
    if (L23 && !BULK) {
        const T L2 = T(L.L2), L3 = T(L.L3);
        // cross-axis part: every site x whose mean difference C_j contains
        // Q(centre).  The branch per site x also keeps the branch-free form
        // to one mean-difference evaluation's reads in flight at a time
        // (without it every read of all seven is hoisted and registers spill).
#pragma unroll
        for (int j = 0; j < 3; ++j) {
#pragma unroll
            for (int s = -1; s <= 1; s += 2) {
                // x = centre - s e_j uses Q(centre) with coefficient a_{j,s}(x)
                int dx, dy, dz;
                unit(j, -s, dx, dy, dz);
                uint32_t mx = P.mask(dx, dy, dz);
                T ap, a0, am;
                mean_diff_coef(mx, j, ap, a0, am);
                const T coef = s > 0 ? ap : am;
                if (coef == T(0)) continue;
                T Ck[3][5], h[5];
                mean_diffs(P, dx, dy, dz, j, mx, Ck);
                cross_h(j, Ck, L2, L3, h);
#pragma unroll
                for (int c = 0; c < 5; ++c) g[c] = fma_t(coef, h[c], g[c]);
            }
            T ap, a0, am;
            mean_diff_coef(m0, j, ap, a0, am);
            if (a0 != T(0)) {
                T Ck[3][5], h[5];
                mean_diffs(P, 0, 0, 0, j, m0, Ck);
                cross_h(j, Ck, L2, L3, h);
#pragma unroll
                for (int c = 0; c < 5; ++c) g[c] = fma_t(a0, h[c], g[c]);
            }
        }
    }
    if (L4) {
        if (L.L4 != 0.0) {
            // chiral term: the site's own tensor, then every C_k(x) holding Q(centre)
            const T hL4 = T(0.5 * L.L4);
            T Cc[3][5], h[5];
            mean_diffs(P, 0, 0, 0, -1, m0, Cc);
            chiral_site(Cc, h);
#pragma unroll
            for (int c = 0; c < 5; ++c) g[c] = fma_t(hL4, h[c], g[c]);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
#pragma unroll
                for (int s = -1; s <= 1; s += 2) {
                    int dx, dy, dz;
                    unit(k, -s, dx, dy, dz);
                    T ap, a0, am;
                    mean_diff_coef(P.mask(dx, dy, dz), k, ap, a0, am);
                    const T coef = s > 0 ? ap : am;
                    if (coef == T(0)) continue;
                    T qx[5];
                    P.load5(dx, dy, dz, qx);
                    chiral_nb(k, qx, h);
#pragma unroll
                    for (int c = 0; c < 5; ++c) g[c] = fma_t(hL4 * coef, h[c], g[c]);
                }
                T ap, a0, am;
                mean_diff_coef(m0, k, ap, a0, am);
                if (a0 != T(0)) {
                    chiral_nb(k, q0, h);
#pragma unroll
                    for (int c = 0; c < 5; ++c) g[c] = fma_t(hL4 * a0, h[c], g[c]);
                }
            }
        }
    }
    // d/dq of 1/2 q^T K q + b^T q = K q + b, K from its upper triangle
    if (!BULK && W == 1 && !(L23 && sizeof(T) == 8) && (m0 & M_ANCH)) {
        T Kq[5];
#pragma unroll
        for (int a = 0; a < 5; ++a) Kq[a] = AR.b[a];
        int t = 0;
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int b = a; b < 5; ++b, ++t) {
                const T k = AR.k[t];
                Kq[a] = fma_t(k, q0[b], Kq[a]);
                if (b != a) Kq[b] = fma_t(k, q0[a], Kq[b]);
            }
#pragma unroll
        for (int c = 0; c < 5; ++c) g[c] += Kq[c];
    }
    if (!BULK && (W == 0 || (L23 && sizeof(T) == 8)) && (m0 & M_ANCH)) {
        // narrow tiles: the row of the FP64 form, read here
        const int at = arow1 - 1;
        if (at >= 0) {
            const double* d = L.anch_data + ANCH_STRIDE * (int64_t)at;
            T Kq[5];
#pragma unroll
            for (int a = 0; a < 5; ++a) Kq[a] = T(d[15 + a]);
            int t = 0;
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int b = a; b < 5; ++b, ++t) {
                    const T k = T(d[t]);
                    Kq[a] = fma_t(k, q0[b], Kq[a]);
                    if (b != a) Kq[b] = fma_t(k, q0[a], Kq[b]);
                }
#pragma unroll
            for (int c = 0; c < 5; ++c) g[c] += Kq[c];
        }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) F[c] = -g[c];
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Block reduction of 4 values in a fixed order: 3 sums and a max
// (LAST_MAX, the step partials), or 4 sums (the energy terms).
template <bool LAST_MAX = true>
__device__ __forceinline__ void block_reduce4(double r[4], double (*scratch)[4]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double a = wave_sum(r[0]), b = wave_sum(r[1]), c = wave_sum(r[2]);
    double d = LAST_MAX ? wave_max(r[3]) : wave_sum(r[3]);
    if (lane == 0) {
        scratch[wv][0] = a; scratch[wv][1] = b; scratch[wv][2] = c; scratch[wv][3] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int w = 0; w < nw; ++w) {
            s0 += scratch[w][0]; s1 += scratch[w][1]; s2 += scratch[w][2];
            s3 = LAST_MAX ? fmax(s3, scratch[w][3]) : s3 + scratch[w][3];
        }
        r[0] = s0; r[1] = s1; r[2] = s2; r[3] = s3;
    }
}

// FIRE controller (Algorithm 1), run by one thread after the grid reduction.
// Steering and restart decided here are applied to v by the next step kernel
// (or by the finalize kernel) as v <- c_v v + c_F F.
__device__ void fire_control(FireDev* st, double P, double nF2, double nv2, double maxF) {
    st->P = P; st->nF2 = nF2; st->nv2 = nv2; st->maxF = maxF;
    if (st->init_pending) {
        st->init_pending = 0;
        if (!(isfinite(nF2) && isfinite(nv2) && isfinite(maxF))) {
            st->status = LQ_NONFINITE; st->done = 1;
        } else if (maxF < st->tol) {
            st->status = LQ_CONVERGED; st->done = 1;
        } else if (st->step >= st->max_steps) {
            st->status = LQ_MAX_STEPS; st->done = 1;
        }
        return;
    }
    st->step += 1;
    st->cur = 1 - st->cur;
    if (!(isfinite(P) && isfinite(nF2) && isfinite(nv2) && isfinite(maxF))) {
        st->status = LQ_NONFINITE;
        st->done = 1;
        st->c_v = 1.0; st->c_F = 0.0;
        return;
    }
    if (st->method != LQ_METHOD_FIRE) {
        // gradient descent and Nesterov: fixed dt and momentum, no steering
    } else if (P > 0.0) {
        double nF = sqrt(nF2), nv = sqrt(nv2);
        st->c_v = 1.0 - st->alpha;
        st->c_F = st->alpha * nv / nF;
        st->n_pos += 1;
        if (st->n_pos > st->n_min) {
            st->dt = fmin(st->dt * st->f_inc, st->dt_max);
            st->alpha = st->alpha * st->f_alpha;
        }
    } else {
        st->c_v = 0.0; st->c_F = 0.0;
        st->dt = st->dt * st->f_dec;
        st->alpha = st->alpha0;
        st->n_pos = 0;
        st->restarts += 1;
    }
    if (maxF < st->tol) {
        st->status = LQ_CONVERGED; st->done = 1;
    } else if (st->step >= st->max_steps) {
        st->status = LQ_MAX_STEPS; st->done = 1;
    } else if (st->step >= st->stop_at) {
        st->done = 1;
    }
}

// Writes this block's partials, and in the last block to arrive reduces all
// of them in block order and runs the controller (the reduction of the FIRE
// initialisation; the step kernels run theirs at the next kernel's start).
__device__ void grid_finish(double r[4], double* partials, FireDev* st, int nblocks, int bid,
                            double (*scratch)[4], int* flag) {
    block_reduce4(r, scratch);
    if (threadIdx.x == 0) {
        double* p = partials + 4 * (int64_t)bid;
        p[0] = r[0]; p[1] = r[1]; p[2] = r[2]; p[3] = r[3];
        __threadfence();
        unsigned t = atomicAdd(&st->ticket, 1u);
        *flag = (t == (unsigned)(nblocks - 1));
    }
    __syncthreads();
    if (!*flag) return;
    __threadfence();
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const volatile double* p = partials + 4 * (int64_t)b;
        s[0] += p[0]; s[1] += p[1]; s[2] += p[2]; s[3] = fmax(s[3], p[3]);
    }
    __syncthreads();
    block_reduce4(s, scratch);
    if (threadIdx.x == 0) {
        // the controller on a register copy of the state: one round trip to
        // read it and one to write it, instead of a chain of dependent
        // global reads (no other block touches the state any more)
        FireDev c = *st;
        fire_control(&c, s[0], s[1], s[2], s[3]);
        c.ticket = 0;
        *st = c;
        __threadfence();
    }
}

// ---------------------------------------------------------------------------
// The z-marching kernel.  MODE_FORCE: F = force(q) only.  MODE_FIRE,
// MODE_GD, MODE_NAG: one fused minimizer step between the two buffers of b:
//   FIRE      v1 = c_v v + c_F F + dt/2 F, q' = q + dt v1, F' = F(q'),
//             v' = v1 + dt/2 F'   (Algorithm 1, steering of the previous step
//             applied first);
//   GD        q' = q + dt F, F' = F(q');
//   Nesterov  m' = mu m + dt F, q' = q + m', F' = F(q' + mu m')  (m in the
//             v buffers; the stencil holds the look-ahead point q' + mu m').
//
// A block owns an X x Y column tile and the planes z0 .. z0+zc-1.  Plane i
// of the march (global z = z0 - 1 + i, i = 0 .. zc+1) is loaded into
// registers (the block's own sites, plus the one-site ring around the tile
// spread over all threads one (site, component) pair at a time), then drifted
// (steering, first half kick, q += dt v) into an LDS slot.  Loads run one
// plane ahead of the drift, so the loads of plane i+1 are in flight while the
// force of plane i-1 is evaluated.
template <typename T, bool L23, int W>
__device__ __forceinline__ void ring_pos(int r, int& px, int& py) {
    constexpr int PX = Tile<T, L23, W>::PX, PY = Tile<T, L23, W>::PY;
    if (r < PX) { px = r; py = 0; }
    else if (r < 2 * PX) { px = r - PX; py = PY - 1; }
    else if (r < 2 * PX + PY - 2) { px = 0; py = r - 2 * PX + 1; }
    else { px = PX - 1; py = r - 2 * PX - (PY - 2) + 1; }
}

// Plane f (1-based within the march) of a chunk takes the bulk evaluation.
__device__ __forceinline__ bool bulk_plane_of(const PlaneBits& b, int f) {
    const int i = f - 1;
    if (i < 0 || i >= CHUNK_MAX) return false;
    const uint64_t w = i < 64 ? b.w[0] : (i < 128 ? b.w[1] : (i < 192 ? b.w[2] : b.w[3]));
    return (w >> (i & 63)) & 1u;
}

#ifndef LQ_PREFETCH
#define LQ_PREFETCH 1
#endif
static_assert(LQ_PREFETCH == 1 || LQ_PREFETCH == 2, "prefetch depth is 1 or 2 planes");

template <typename T, bool L23, bool L4, int MODE, bool BULK, int W>
__device__ __forceinline__ void march(const LatDev& L, const T* __restrict__ q_in,
                                      const T* __restrict__ v_in, const T* __restrict__ F_in,
                                      T* __restrict__ q_out, T* __restrict__ v_out,
                                      T* __restrict__ F_out, T cv, T cF, T dt, T hdt, int x0, int y0,
                                      int z0, int zc, T (*sq)[5][Tile<T, L23, W>::PY][Tile<T, L23, W>::PX],
                                      uint8_t (*sm)[Tile<T, L23, W>::PY][Tile<T, L23, W>::PX], double red[4],
                                      const PlaneBits plane_bulk) {
    using G = Tile<T, L23, W>;
    constexpr int NS = 4;
    constexpr int PF = LQ_PREFETCH;  // planes of raw data in flight
    constexpr int TX = G::X, NTHREADS = G::N, RING = G::RING;
    constexpr int RING_ITEMS = G::RING_ITEMS, ITEMS_PER_THREAD = G::IPT;
    constexpr bool STEP = MODE != MODE_FORCE;
    constexpr bool USES_V = MODE == MODE_FIRE || MODE == MODE_NAG;
    constexpr bool ZERO_SOLID = !BULK && L23 && branch_free<T>();
    const int64_t N = L.N;
    const int nxy = L.nx * L.ny;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own_xy = gx < L.nx && gy < L.ny;
    int sxy_own;
    {
        const int wx = wrapc(gx, L.nx, L.per[0]), wy = wrapc(gy, L.ny, L.per[1]);
        sxy_own = (wx >= 0 && wy >= 0) ? wx + L.nx * wy : -1;
    }
    // ring items of this thread
    int it_c[ITEMS_PER_THREAD], it_px[ITEMS_PER_THREAD], it_py[ITEMS_PER_THREAD], it_sxy[ITEMS_PER_THREAD];
#pragma unroll
    for (int j = 0; j < ITEMS_PER_THREAD; ++j) {
        const int k = threadIdx.x + j * NTHREADS;
        it_c[j] = -1; it_px[j] = 0; it_py[j] = 0; it_sxy[j] = -1;
        if (k < RING_ITEMS) {
            it_c[j] = k / RING;
            ring_pos<T, L23, W>(k % RING, it_px[j], it_py[j]);
            const int wx = wrapc(x0 - 1 + it_px[j], L.nx, L.per[0]);
            const int wy = wrapc(y0 - 1 + it_py[j], L.ny, L.per[1]);
            it_sxy[j] = (wx >= 0 && wy >= 0) ? wx + L.nx * wy : -1;
        }
    }
    // raw data of a plane still to drift (PF planes are in flight)
    struct Raw {
        T q[5], v[5], f[5];
        T iq[ITEMS_PER_THREAD], iv[ITEMS_PER_THREAD], iF[ITEMS_PER_THREAD];
        uint32_t m, im[ITEMS_PER_THREAD];
    };

    const uint32_t cs = (uint32_t)N * (uint32_t)sizeof(T);  // bytes per component
    const uint32_t fb = 5u * cs;                               // bytes per field
    const __amdgpu_buffer_rsrc_t rq_in = field_rsrc(q_in, fb);
    const __amdgpu_buffer_rsrc_t rv_in = field_rsrc(USES_V ? v_in : q_in, fb);
    const __amdgpu_buffer_rsrc_t rF_in = field_rsrc(STEP ? F_in : q_in, fb);
    const __amdgpu_buffer_rsrc_t rq_out = field_rsrc(STEP ? q_out : F_out, fb);
    const __amdgpu_buffer_rsrc_t rv_out = field_rsrc(USES_V ? v_out : F_out, fb);
    const __amdgpu_buffer_rsrc_t rF_out = field_rsrc(F_out, fb);
    const __amdgpu_buffer_rsrc_t rmask = field_rsrc(L.mask, (uint32_t)N);
    constexpr uint32_t NONE = 0xFFFFFFFFu;  // past every resource: loads give 0, stores drop
    // Branch-free loads: an invalid position gets an offset past the end of the
    // buffer instead of a branch, so the wait counts stay exact and the stores
    // of the previous plane can drain while this plane is drifted.
    auto load = [&](int i, Raw& R) {
        const int wz = (i >= 0 && i <= zc + 1) ? wrapc(z0 - 1 + i, L.nz, L.per[2]) : -1;
        const bool ok = sxy_own >= 0 && wz >= 0;
        const uint32_t site = (uint32_t)(sxy_own + nxy * wz);
        const uint32_t off = ok ? site * (uint32_t)sizeof(T) : NONE;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            R.q[c] = bld<T>(rq_in, off, c * cs);
            if (USES_V) R.v[c] = bld<T>(rv_in, off, c * cs);
            if (STEP) R.f[c] = bld<T>(rF_in, off, c * cs);
        }
        if (!BULK) R.m = __builtin_amdgcn_raw_buffer_load_b8(rmask, (int)(ok ? site : NONE), 0, 0);
#pragma unroll
        for (int j = 0; j < ITEMS_PER_THREAD; ++j) {
            const bool okj = it_sxy[j] >= 0 && wz >= 0;
            const uint32_t t = (uint32_t)(it_sxy[j] + nxy * wz);
            const uint32_t offj = okj ? ((uint32_t)it_c[j] * (uint32_t)N + t) * (uint32_t)sizeof(T) : NONE;
            R.iq[j] = bld<T>(rq_in, offj, 0u);
            if (USES_V) R.iv[j] = bld<T>(rv_in, offj, 0u);
            if (STEP) R.iF[j] = bld<T>(rF_in, offj, 0u);
            // the branch-free kernels zero the sites that are not simulated,
            // so they need the mask of every ring item
            if (!BULK) R.im[j] = __builtin_amdgcn_raw_buffer_load_b8(rmask, (int)(okj && (ZERO_SOLID || it_c[j] == 0) ? t : NONE), 0, 0);
        }
    };
    // drift the registers into LDS slot; returns the own site's q' and v1
    // (FIRE: v after the first half kick; Nesterov: m')
    auto drift = [&](const Raw& R, int slot, T qn[5], T v1[5], uint32_t& m) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            T x;
            if (MODE == MODE_FIRE) {
                const T vm = fma_t(cv, R.v[c], cF * R.f[c]);
                v1[c] = fma_t(hdt, R.f[c], vm);
                qn[c] = fma_t(dt, v1[c], R.q[c]);
                x = qn[c];
            } else if (MODE == MODE_GD) {
                qn[c] = fma_t(dt, R.f[c], R.q[c]);
                v1[c] = T(0);
                x = qn[c];
            } else if (MODE == MODE_NAG) {
                v1[c] = fma_t(cv, R.v[c], dt * R.f[c]);
                qn[c] = R.q[c] + v1[c];
                x = fma_t(cv, v1[c], qn[c]);
            } else {
                qn[c] = R.q[c];
                v1[c] = T(0);
                x = qn[c];
            }
            // branch-free kernels: a site that is not simulated holds 0 in
            // LDS, whatever its stored tensor (the force reads it with weight 0)
            if (ZERO_SOLID) x = (R.m & M_SIM) ? x : T(0);
            sq[slot][c][ty + 1][tx + 1] = x;
        }
        m = BULK ? (uint32_t)M_FULL : R.m;
        if (!BULK) sm[slot][ty + 1][tx + 1] = (uint8_t)R.m;
#pragma unroll
        for (int j = 0; j < ITEMS_PER_THREAD; ++j) {
            if (it_c[j] < 0) continue;
            T x = R.iq[j];
            if (MODE == MODE_FIRE) {
                const T vm = fma_t(cv, R.iv[j], cF * R.iF[j]);
                x = fma_t(dt, fma_t(hdt, R.iF[j], vm), x);
            } else if (MODE == MODE_GD) {
                x = fma_t(dt, R.iF[j], x);
            } else if (MODE == MODE_NAG) {
                const T mj = fma_t(cv, R.iv[j], dt * R.iF[j]);
                x = fma_t(cv, mj, x + mj);
            }
            if (ZERO_SOLID) x = (R.im[j] & M_SIM) ? x : T(0);
            sq[slot][it_c[j]][it_py[j]][it_px[j]] = x;
            if (!BULK && it_c[j] == 0) sm[slot][it_py[j]][it_px[j]] = (uint8_t)R.im[j];
        }
    };
    auto slot_of = [](int i) { return (i + NS) & (NS - 1); };

    // Loads run one plane ahead: iteration j drifts plane j (loaded during
    // iteration j-1), issues the loads of plane j+1, and evaluates and stores
    // the force of plane j-1 from the LDS planes j-2 .. j.  Every path into
    // the drift has the same stores queued behind the loads it waits for
    // (the prologue stores to an offset past the end of the buffers, which
    // the hardware drops), so the wait lets those stores drain.  Planes
    // outside 0 .. zc+1 load from out-of-range offsets; forces outside
    // 1 .. zc are stored nowhere.
    // v1 and mask of the own site: `older` is the plane whose force is
    // evaluated in this iteration, `newer` the plane just drifted.
    T v1_older[5], v1_newer[5], q_older[5], q_newer[5];
    uint32_t m_older = 0, m_newer = 0;
    // anchoring row (1 + row, 0: none) of the own site: loaded right after
    // the drift, once the mask is known, so that it has arrived by the time
    // the force of that plane is evaluated in the next iteration
    const __amdgpu_buffer_rsrc_t ranch = field_rsrc(L.anch_index, (uint32_t)N * 4u);
    int a_older = 0, a_newer = 0;
#pragma unroll
    for (int c = 0; c < 5; ++c) { v1_older[c] = T(0); v1_newer[c] = T(0); q_older[c] = T(0); q_newer[c] = T(0); }
    // One iteration of the march: drift plane j from R (loaded PF iterations
    // earlier), reload R with plane j + PF, and evaluate and store the force of
    // plane j - 1 from the LDS planes j - 2 .. j.
    T fmax_abs = T(0);  // max |F| in the field's own type (exact), folded into red[3] at the end
    auto plane = [&](int j, Raw& R) {
        if (!L23) __builtin_amdgcn_s_setprio(0);  // drift and loads at the normal priority
        // anchoring forms of plane j - 1, whose force this iteration
        // evaluates.  Wide tiles issue them first, so that they arrive while
        // plane j is drifted and the block meets at the barrier.  Narrow tiles
        // (the small boxes of a batch) read the FP64 rows inside the force
        // instead: on a stream of small boxes the early loads raised the tail
        // latency.  So do the FP64 L2/L3 kernels (registers; see site_force).
        AnchRow<T> A;
        if (!BULK && W == 1 && !(L23 && sizeof(T) == 8)) {
            const int f = j - 1;
            const bool bulk_plane = bulk_plane_of(plane_bulk, f);
            // only waves with an anchored site issue the loads
            if (!bulk_plane && __builtin_amdgcn_ballot_w64((m_newer & M_ANCH) != 0) != 0)
                anch_load(L, (m_newer & M_ANCH) ? a_newer : 0, A);
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) { v1_older[c] = v1_newer[c]; q_older[c] = q_newer[c]; }
        m_older = m_newer;
        a_older = a_newer;
        drift(R, slot_of(j), q_newer, v1_newer, m_newer);
        if (!BULK) {
            const bool anch = own_xy && j >= 1 && j <= zc && (m_newer & M_ANCH);
            const uint32_t sj = (uint32_t)(gx + L.nx * gy + nxy * (z0 + j - 1));
            a_newer = (int)__builtin_amdgcn_raw_buffer_load_b32(ranch, (int)(anch ? sj * 4u : NONE), 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
        load(j + PF, R);
        __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of this plane's stores
        lds_barrier();
        // one-constant kernels: waves past the barrier (force and stores) go
        // before waves still drifting, so each plane's stores leave sooner
        // (measured 0.7% on the 256^3 multi-colloid step; not for L2/L3)
        if (!L23) __builtin_amdgcn_s_setprio(1);
        {
            const int f = j - 1;  // plane whose force is evaluated
            const bool in_chunk = f >= 1;
            const int s = gx + L.nx * gy + nxy * (z0 + f - 1);
            const uint32_t off = (own_xy && in_chunk) ? (uint32_t)s * (uint32_t)sizeof(T) : NONE;
            const bool live = own_xy && in_chunk && (m_older & M_SIM);
            Stencil<T, L23, BULK, W> P;
            P.q = sq; P.m = sm;
            P.s[0] = slot_of(f - 1); P.s[1] = slot_of(f); P.s[2] = slot_of(f + 1);
            P.cx = tx + 1; P.cy = ty + 1;
            T F[5];
            // a plane whose 3 x 3 x 3 neighbourhoods are all full bulk sites
            // takes the bulk evaluation also inside a boundary tile (wide
            // tiles only: the narrow ones serve small boxes, where few planes
            // qualify and the extra code costs registers).  The first two
            // iterations have no plane of the chunk to evaluate (their stores
            // are dropped): the L2/L3 kernels compute no force there (in the
            // one-constant kernels the branch split the loop body and measured
            // 3% slower than the two wasted evaluations).
            if (L23 && !in_chunk) {
#pragma unroll
                for (int c = 0; c < 5; ++c) F[c] = T(0);
            } else if (W == 1 && !BULK && bulk_plane_of(plane_bulk, f)) {
                Stencil<T, L23, true, W> PB;
                PB.q = sq; PB.m = sm;
                PB.s[0] = P.s[0]; PB.s[1] = P.s[1]; PB.s[2] = P.s[2];
                PB.cx = P.cx; PB.cy = P.cy;
                site_force<T, L23, L4, true, W>(PB, (uint32_t)M_FULL, L, A, 0, F);
            } else {
                site_force<T, L23, L4, BULK, W>(P, m_older, L, A, a_older, F);
            }
            {
                constexpr int POL = store_policy<T, L23>();
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const T Fc = live ? F[c] : T(0);
                    if (MODE == MODE_FIRE || MODE == MODE_NAG) {
                        const T v2 = live ? (MODE == MODE_FIRE ? fma_t(hdt, F[c], v1_older[c]) : v1_older[c]) : T(0);
                        const T qc = live ? (MODE == MODE_FIRE ? P.at(0, 0, 0, c) : q_older[c]) : T(0);
                        bst_p<T, POL>(rq_out, off, c * cs, qc);
                        bst_p<T, POL>(rv_out, off, c * cs, v2);
                        bst_p<T, POL>(rF_out, off, c * cs, Fc);
                        const double fd = (double)Fc, vd = (double)v2;
                        red[0] = fma(fd, vd, red[0]);
                        red[1] = fma(fd, fd, red[1]);
                        red[2] = fma(vd, vd, red[2]);
                        fmax_abs = fmax(fmax_abs, fabs(Fc));
                    } else if (MODE == MODE_GD) {
                        const T qc = live ? P.at(0, 0, 0, c) : T(0);
                        bst_p<T, POL>(rq_out, off, c * cs, qc);
                        bst_p<T, POL>(rF_out, off, c * cs, Fc);
                        const double fd = (double)Fc;
                        red[1] = fma(fd, fd, red[1]);
                        fmax_abs = fmax(fmax_abs, fabs(Fc));
                    } else {
                        bst_p<T, POL>(rF_out, off, c * cs, Fc);
                    }
                }
            }
        }
    };
    Raw RA, RB;
    load(0, RA);
    if (PF == 2) load(1, RB);
    __builtin_amdgcn_sched_barrier(0);  // keep the dropped stores behind the loads
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        bst_p<T, 2>(rF_out, NONE, c * cs, T(0));
        if (STEP) bst_p<T, 2>(rq_out, NONE, c * cs, T(0));
        if (USES_V) bst_p<T, 2>(rv_out, NONE, c * cs, T(0));
    }
    __builtin_amdgcn_sched_barrier(0);
    if (PF == 1) {
#pragma clang loop unroll(disable)
        for (int j = 0; j <= zc + 1; ++j) plane(j, RA);
    } else {
#pragma clang loop unroll(disable)
        for (int j = 0; j <= zc + 1; j += 2) {
            plane(j, RA);
            if (j + 1 <= zc + 1) plane(j + 1, RB);
        }
    }
    red[3] = fmax(red[3], (double)fmax_abs);
}

// Sums the partials of nblocks blocks in block order (every block of a
// kernel that calls this gets the same sums: they depend on the block size
// and nblocks only).
__device__ __forceinline__ void sum_partials(const double* partials, int nblocks, double s[4],
                                             double (*scratch)[4]) {
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const double* p = partials + 4 * (int64_t)b;
        s[0] += p[0]; s[1] += p[1]; s[2] += p[2]; s[3] = fmax(s[3], p[3]);
    }
    __syncthreads();
    block_reduce4(s, scratch);
}

// Start of step kernel k (1-based within a call) of a lattice: the
// controller on the reduction of step k - 1, in every block (the same sums
// in the same order give every block the same result), so that no block
// waits for a last one to finish the previous kernel.  Block 0 keeps the
// new state in st[(k - 1) & 1].  Returns true (every thread) when the run has
// stopped; the step's parameters go to cd (dt, c_v, c_F, mu) and ci (cur,
// stop; ci[2] takes the stop word).
__device__ bool dc_begin(FireDev* st, const double* partials, int nblocks, int k, int bid,
                         double (*scratch)[4], double* cd, int* ci) {
    DcCtl* ctl = (DcCtl*)(st + 2);
    // one read of the stop word per block: waves that read it apart could see
    // different values while block 0 of this kernel sets it
    if (threadIdx.x == 0) ci[2] = ((volatile const DcCtl*)ctl)->halt;
    __syncthreads();
    if (ci[2]) return true;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (k >= 2) sum_partials(partials + 4 * (int64_t)((k - 1) & 1) * nblocks, nblocks, s, scratch);
    if (threadIdx.x == 0) {
        FireDev c = st[k >= 2 ? (k & 1) : 0];
        if (k >= 2 && !c.done) fire_control(&c, s[0], s[1], s[2], s[3]);
        const int stop = c.done ? 1 : 0;
        if (bid == 0) {
            if (k >= 2) st[(k - 1) & 1] = c;
            if (stop) {
                ctl->slot = k >= 2 ? ((k - 1) & 1) : 0;
                ctl->halt = 1;
            }
        }
        cd[0] = c.dt; cd[1] = c.c_v; cd[2] = c.c_F; cd[3] = c.mu;
        ci[0] = c.cur; ci[1] = stop;
    }
    __syncthreads();
    return ci[1] != 0;
}

// One block of the force / FIRE step: tile `bid` of lattice L.  `nblocks`
// is the lattice's own tile count; partials are indexed by tile, so the
// reduction order does not depend on how blocks are dispatched.  The
// controller of step k - 1 runs at the start (dc_begin); the partials of
// step k go to slot k & 1.
template <typename T, bool L23, bool L4, int MODE, int W>
__device__ __forceinline__ void step_block(const LatDev& L, const Bufs<T>& b, const T* __restrict__ qin,
                                           T* __restrict__ Fout, double* partials, FireDev* st,
                                           int nblocks, int bid, int k) {
    constexpr int NS = 4;
    using G = Tile<T, L23, W>;
    constexpr int PX = G::PX, PY = G::PY;
    __shared__ T sq[NS][5][PY][PX];
    __shared__ uint8_t sm[NS][PY][PX];
    __shared__ double scratch[G::N / 64][4];
    __shared__ double ctl_d[4];
    __shared__ int ctl_i[3];

    constexpr bool STEP = MODE != MODE_FORCE;
    const T *q_in, *v_in = nullptr, *F_in = nullptr;
    T *q_out = nullptr, *v_out = nullptr, *F_out;
    T cv = T(1), cF = T(0), dt = T(0), hdt = T(0);
    if (STEP) {
        if (dc_begin(st, partials, nblocks, k, bid, scratch, ctl_d, ctl_i)) return;
        const int cur = ctl_i[0];
        const double dtd = ctl_d[0], c_v = ctl_d[1], c_F = ctl_d[2], mu = ctl_d[3];
        // selects rather than indexing by cur, which would put b in scratch
        q_in = cur ? b.q[1] : b.q[0]; v_in = cur ? b.v[1] : b.v[0]; F_in = cur ? b.F[1] : b.F[0];
        q_out = cur ? b.q[0] : b.q[1]; v_out = cur ? b.v[0] : b.v[1]; F_out = cur ? b.F[0] : b.F[1];
        dt = T(dtd); hdt = T(0.5 * dtd);
        if (MODE == MODE_FIRE) { cv = T(c_v); cF = T(c_F); }
        if (MODE == MODE_NAG) cv = T(mu);
    } else {
        q_in = qin;
        F_out = Fout;
    }
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    // the block's chunks one after the other: a packed plan (FP64 L2/L3 only)
    // gives some blocks two; every other plan one per block, chunk bid (the
    // loop costs the other kernels registers)
    constexpr bool PACKED = L23 && sizeof(T) == 8;
    const int i0 = PACKED ? L.first[bid] : bid, i1 = PACKED ? L.first[bid + 1] : bid + 1;
    for (int i = i0; i < i1; ++i) {
        if (i > i0) __syncthreads();  // every wave is done with the LDS planes of the previous chunk
        const Chunk ch = L.chunks[i];
        const int x0 = ch.x0, y0 = ch.y0, z0 = ch.z0, zc = ch.zc;
        if (L.tile_bulk[i]) {
            PlaneBits all;
#pragma unroll
            for (int w = 0; w < PLANE_WORDS; ++w) all.w[w] = ~(uint64_t)0;
            march<T, L23, L4, MODE, true, W>(L, q_in, v_in, F_in, q_out, v_out, F_out, cv, cF, dt, hdt, x0, y0, z0,
                                             zc, sq, sm, red, all);
        } else {
            march<T, L23, L4, MODE, false, W>(L, q_in, v_in, F_in, q_out, v_out, F_out, cv, cF, dt, hdt, x0, y0, z0,
                                              zc, sq, sm, red, L.tile_planes[i]);
        }
    }
    if (STEP) {
        block_reduce4(red, scratch);
        if (threadIdx.x == 0) {
            double* p = partials + 4 * ((int64_t)(k & 1) * nblocks + bid);
            p[0] = red[0]; p[1] = red[1]; p[2] = red[2]; p[3] = red[3];
        }
    }
}

// After the k_steps step kernels of a call: the controller on the last
// step's reduction (the same sums, in the same order, as in a step kernel
// of NT threads), or the state the run stopped with, into st[0].
template <int NT>
__device__ void dc_final(FireDev* st, const double* partials, int nblocks, int k_steps, double (*scratch)[4]) {
    DcCtl* ctl = (DcCtl*)(st + 2);
    if (ctl->halt) {
        if (threadIdx.x == 0) {
            const int sl = ctl->slot;
            if (sl != 0) st[0] = st[sl];
            ctl->halt = 0;
        }
        return;
    }
    if (k_steps <= 0) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    sum_partials(partials + 4 * (int64_t)(k_steps & 1) * nblocks, nblocks, s, scratch);
    if (threadIdx.x == 0) {
        FireDev c = st[k_steps >= 2 ? ((k_steps - 1) & 1) : 0];
        fire_control(&c, s[0], s[1], s[2], s[3]);
        st[0] = c;
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_dc_control(FireDev* st, const double* partials, int nblocks, int k_steps) {
    __shared__ double scratch[NT / 64][4];
    dc_final<NT>(st, partials, nblocks, k_steps, scratch);
}

// The same for every member of a batch group (one block per member).
template <int NT>
__global__ __launch_bounds__(NT) void k_batch_dc_control(const MemberDev* __restrict__ mem, int k_steps) {
    __shared__ double scratch[NT / 64][4];
    const MemberDev& M = mem[blockIdx.x];
    dc_final<NT>(M.st, M.partials, M.nblocks, k_steps, scratch);
}

// L4: the kernel evaluates the chiral term (a kernel of its own, so that the
// common L2/L3 kernels do not carry its registers).  TWO: held to two waves
// per SIMD (the FP64 L2/L3 kernel for lattices whose one-wave chunks would be
// short; LatDev::two_waves).
template <typename T, bool L23, bool L4, int MODE, int W, bool TWO = false>
__global__ __launch_bounds__((Tile<T, L23, W>::N)) __attribute__((amdgpu_waves_per_eu(L4 ? 1 : (TWO ? 2 : Tile<T, L23, W>::WAVES)))) void k_march(LatDev L, Bufs<T> b, const T* __restrict__ qin,
                                                    T* __restrict__ Fout, double* partials,
                                                    FireDev* st, int k) {
    const int nblocks = (int)gridDim.x;
    int bid = (int)blockIdx.x;
    // keep neighbouring tiles on one XCD: dispatch is round-robin over 8
    // XCDs, so XCD x runs the blocks x, x + 8, ...; they take the x-th
    // contiguous share of the plan (the first nblocks % 8 shares one longer)
    {
        const int x = bid & 7, q = nblocks >> 3, r = nblocks & 7;
        bid = x * q + (x < r ? x : r) + (bid >> 3);
    }
    step_block<T, L23, L4, MODE, W>(L, b, qin, Fout, partials, st, nblocks, bid, k);
}

// ---------------------------------------------------------------------------
// Batched steps: one launch advances every member of a batch of lattices by
// one FIRE step.  Block b belongs to the member m with off[m] <= b <
// off[m+1]; each member keeps its own controller, partials and ticket, so
// its trajectory is bit for bit the one it has alone.
__device__ __forceinline__ int member_of(const int* __restrict__ off, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T, bool L23, int W>
__global__ __launch_bounds__((Tile<T, L23, W>::N)) __attribute__((amdgpu_waves_per_eu(Tile<T, L23, W>::WAVES))) void k_march_batch(const MemberDev* __restrict__ mem,
                                                          const int* __restrict__ off, int n_members, int k) {
    const int m = member_of(off, n_members, (int)blockIdx.x);
    const MemberDev& M = mem[m];
    Bufs<T> b;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        b.q[i] = (T*)M.q[i]; b.v[i] = (T*)M.v[i]; b.F[i] = (T*)M.F[i];
    }
    const LatDev& L = M.L;
    step_block<T, L23, L23, MODE_FIRE, W>(L, b, nullptr, nullptr, M.partials, M.st, M.nblocks,
                                          (int)blockIdx.x - off[m], k);
}

__global__ void k_batch_begin(const MemberDev* __restrict__ mem, int n_members, int64_t n_steps) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_members) return;
    FireDev* st = mem[m].st;
    ((DcCtl*)(st + 2))->halt = 0;
    if (st->status == LQ_RUNNING) {
        st->done = 0;
        st->stop_at = st->step + n_steps;
        if (n_steps <= 0) st->done = 1;
    }
}

// State of every member into its buffer 0 with pending steering applied.
template <typename T>
__global__ __launch_bounds__(256) void k_batch_finalize(const MemberDev* __restrict__ mem,
                                                        const int* __restrict__ off, int n_members) {
    const int m = member_of(off, n_members, (int)blockIdx.x);
    const MemberDev& M = mem[m];
    const FireDev* st = M.st;
    const int cur = st->cur;
    const T cv = T(st->c_v), cF = T(st->c_F);
    const int64_t n = 5 * M.L.N;
    const int nb = off[m + 1] - off[m];
    T* q0 = (T*)M.q[0]; T* v0 = (T*)M.v[0]; T* F0 = (T*)M.F[0];
    const T* qc = (const T*)M.q[cur]; const T* vc = (const T*)M.v[cur]; const T* Fc = (const T*)M.F[cur];
    for (int64_t i = ((int)blockIdx.x - off[m]) * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)nb * blockDim.x) {
        const T v = vc[i], f = Fc[i];
        const T vm = fma_t(cv, v, cF * f);
        if (cur) { q0[i] = qc[i]; F0[i] = f; }
        v0[i] = vm;
    }
}

// Resets the pending steering of every member and gathers the controller
// states into one array for a single copy to the host.
__global__ void k_batch_reset_gather(const MemberDev* __restrict__ mem, int n_members, FireDev* out) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_members) return;
    FireDev* st = mem[m].st;
    st->cur = 0;
    st->c_v = 1.0;
    st->c_F = 0.0;
    out[m] = *st;
}

// ---------------------------------------------------------------------------
// lq_fire_init reduction: |F|^2, |v|^2, F.v, max|F_i| of the initial state,
// then the controller's initial convergence test.
template <typename T>
__global__ __launch_bounds__(256) void k_init_reduce(const T* __restrict__ F, const T* __restrict__ v,
                                                     int64_t n, double* partials, FireDev* st) {
    __shared__ double scratch[4][4];
    __shared__ int last_flag;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double f = (double)F[i], w = v ? (double)v[i] : 0.0;
        r[0] = fma(f, w, r[0]);
        r[1] = fma(f, f, r[1]);
        r[2] = fma(w, w, r[2]);
        r[3] = fmax(r[3], fabs(f));
        if (f != f) r[3] = f;
    }
    grid_finish(r, partials, st, (int)gridDim.x, (int)blockIdx.x, scratch, &last_flag);
}

__global__ void k_begin(FireDev* st, int64_t n_steps) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ((DcCtl*)(st + 2))->halt = 0;
        if (st->status == LQ_RUNNING) {
            st->done = 0;
            st->stop_at = st->step + n_steps;
            if (n_steps <= 0) st->done = 1;
        }
    }
}

// Brings the current state into buffer 0 and applies the pending steering.
// Gradient descent leaves v untouched (with_v = false).
template <typename T>
__global__ __launch_bounds__(256) void k_finalize(Bufs<T> b, int64_t n, const FireDev* st, int with_v) {
    const int cur = st->cur;
    const T cv = T(st->c_v), cF = T(st->c_F);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T f = b.F[cur][i];
        if (cur) {
            b.q[0][i] = b.q[1][i];
            b.F[0][i] = f;
        }
        if (with_v) b.v[0][i] = fma_t(cv, b.v[cur][i], cF * f);
    }
}

// y = q + mu m: the Nesterov look-ahead point of a resumed state.
template <typename T>
__global__ __launch_bounds__(256) void k_lookahead(const T* __restrict__ q, const T* __restrict__ m, T mu,
                                                   T* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = fma_t(mu, m[i], q[i]);
}

__global__ void k_reset_mix(FireDev* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->cur = 0;
        st->c_v = 1.0;
        st->c_F = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t* p, int64_t n_words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// q = 3/2 S (n n - I/3) at simulated sites, 0 inside objects.  Products are
// rounded one by one (no contraction) so that the state is reproducible.
template <typename T>
__global__ __launch_bounds__(256) void k_uniaxial(LatDev L, const double* __restrict__ dirs, double S,
                                                  T* __restrict__ q) {
#pragma clang fp contract(off)
    const int64_t N = L.N;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N;
         s += (int64_t)gridDim.x * blockDim.x) {
        double r[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (L.mask[s] & M_SIM) {
            double nx = dirs[s], ny = dirs[N + s], nz = dirs[2 * N + s];
            double h = 1.5 * S;
            r[0] = h * (nx * nx - 1.0 / 3.0);
            r[1] = h * nx * ny;
            r[2] = h * nx * nz;
            r[3] = h * (ny * ny - 1.0 / 3.0);
            r[4] = h * ny * nz;
        }
        for (int c = 0; c < 5; ++c) q[c * N + s] = T(r[c]);
    }
}

// ---------------------------------------------------------------------------
// Energy: one thread per site, FP64 arithmetic, per-term block partials
// reduced in block order by the last block.
template <typename T, bool L23>
__global__ __launch_bounds__(256) void k_energy(LatDev L, const T* __restrict__ q, double* partials,
                                                EnergyOut* out, uint32_t* ticket) {
    __shared__ double scratch[4][4];
    __shared__ int last_flag;
    const int64_t N = L.N;
    double e_b = 0.0, e_d = 0.0, e_a = 0.0, e_x = 0.0;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N;
         s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t m = L.mask[s];
        if (!(m & M_SIM)) continue;
        const int x = (int)(s % L.nx), y = (int)((s / L.nx) % L.ny), z = (int)(s / ((int64_t)L.nx * L.ny));
        double q0[5];
        for (int c = 0; c < 5; ++c) q0[c] = (double)q[c * N + s];
        double Q[3][3];
        full_of(q0, Q);
        double t2 = 0.0, t3 = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                t2 += Q[i][j] * Q[j][i];
                for (int k = 0; k < 3; ++k) t3 += Q[i][j] * Q[j][k] * Q[k][i];
            }
        e_b += 0.5 * L.A * t2 + L.B / 3.0 * t3 + 0.25 * L.C * t2 * t2;
        // neighbour q along each axis and direction
        double qn[3][2][5];
        for (int k = 0; k < 3; ++k)
            for (int si = 0; si < 2; ++si) {
                const int sg = si == 0 ? 1 : -1;
                for (int c = 0; c < 5; ++c) qn[k][si][c] = 0.0;
                if (!has_nb(m, k, sg)) continue;
                int c3[3] = {x, y, z};
                const int n3[3] = {L.nx, L.ny, L.nz};
                c3[k] = wrapc(c3[k] + sg, n3[k], L.per[k]);
                const int64_t t = (int64_t)c3[0] + (int64_t)L.nx * ((int64_t)c3[1] + (int64_t)L.ny * c3[2]);
                for (int c = 0; c < 5; ++c) qn[k][si][c] = (double)q[c * N + t];
            }
        double ed = 0.0;
        double Cm[3][5];
        for (int k = 0; k < 3; ++k) {
            const int nk = n_choices(m, k);
            double acc1 = 0.0, acc23 = 0.0;
            for (int si = 0; si < 2; ++si) {
                if (!has_nb(m, k, si == 0 ? 1 : -1)) continue;
                double d[5], o[5];
                for (int c = 0; c < 5; ++c) d[c] = qn[k][si][c] - q0[c];
                metric(d, o);
                for (int c = 0; c < 5; ++c) acc1 += d[c] * o[c];
                if (L23) {
                    column_metric(k, d, o);
                    for (int c = 0; c < 5; ++c) acc23 += d[c] * o[c];
                }
            }
            if (nk > 0) {
                ed += 0.5 * L.L1 * acc1 / nk;
                if (L23) ed += 0.5 * (L.L2 + L.L3) * acc23 / nk;
            }
            double ap, a0, am;
            mean_diff_coef(m, k, ap, a0, am);
            for (int c = 0; c < 5; ++c)
                Cm[k][c] = ap * qn[k][0][c] + a0 * q0[c] + am * qn[k][1][c];
        }
        if (L23) {
            // sum_{j<k} L2 sum_i C_j,ij C_k,ik + L3 sum_i C_j,ik C_k,ij
            double Cf[3][3][3];
            for (int k = 0; k < 3; ++k) full_of(Cm[k], Cf[k]);
            for (int j = 0; j < 3; ++j)
                for (int k = j + 1; k < 3; ++k)
                    for (int i = 0; i < 3; ++i)
                        ed += L.L2 * Cf[j][i][j] * Cf[k][i][k] + L.L3 * Cf[j][i][k] * Cf[k][i][j];
            // chiral term L4/2 eps_lik Q_lj C_k,ij
            double e4 = 0.0;
            for (int l = 0; l < 3; ++l)
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) {
                        if (eps3(l, i, k) == 0) continue;
                        for (int j = 0; j < 3; ++j) e4 += eps3(l, i, k) * Q[l][j] * Cf[k][i][j];
                    }
            ed += 0.5 * L.L4 * e4;
        }
        e_d += ed;
        double qe = 0.0;
        for (int c = 0; c < 5; ++c) qe += L.ext[c] * q0[c];
        e_x -= qe;
        if (m & M_ANCH) {
            const int at = L.anch_index[s] - 1;
            if (at >= 0) {
                // 1/2 q^T K q + b^T q + c
                const double* d = L.anch_data + ANCH_STRIDE * (int64_t)at;
                double quad = 0.0, lin = 0.0;
                int t = 0;
                for (int a = 0; a < 5; ++a) {
                    lin += d[15 + a] * q0[a];
                    for (int b = a; b < 5; ++b, ++t)
                        quad += (b == a ? 0.5 : 1.0) * d[t] * q0[a] * q0[b];
                }
                e_a += quad + lin + d[20];
            }
        }
    }
    double r[4] = {e_b, e_d, e_a, e_x};
    block_reduce4<false>(r, scratch);
    if (threadIdx.x == 0) {
        double* p = partials + 4 * (int64_t)blockIdx.x;
        p[0] = r[0]; p[1] = r[1]; p[2] = r[2]; p[3] = r[3];
        __threadfence();
        unsigned t = atomicAdd(ticket, 1u);
        last_flag = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last_flag) return;
    __threadfence();
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) {
        const volatile double* p = partials + 4 * (int64_t)b;
        s4[0] += p[0]; s4[1] += p[1]; s4[2] += p[2]; s4[3] += p[3];
    }
    __syncthreads();
    block_reduce4<false>(s4, scratch);
    if (threadIdx.x == 0) {
        out->bulk = s4[0]; out->elastic = s4[1]; out->anch = s4[2]; out->ext = s4[3];
        *ticket = 0;
        __threadfence();
    }
}

// ---------------------------------------------------------------------------
// Director and defect extraction (Eq. Qtensor and the text after it; the
// display of directors and defects in sec. IV): per simulated site the
// largest eigenvalue of Q and its eigenvector, and whether that eigenvalue
// lies below a threshold.  FP64 arithmetic.  For a traceless symmetric Q
// with p = sqrt(tr(Q^2)/6) the eigenvalues are 2p cos((acos(r) + 2 pi m)/3),
// r = det(Q)/(2 p^3) (the trigonometric solution of the characteristic
// cubic), m = 0 giving the largest.  The eigenvector is the largest cross
// product of two rows of Q - lambda I; when Q - lambda I has rank one (the
// largest eigenvalue is doubly degenerate) any vector normal to its
// non-zero row is an eigenvector.  n and -n being equal, the sign makes the
// largest-magnitude component positive.
template <typename T>
__global__ __launch_bounds__(256) void k_directors(LatDev L, const T* __restrict__ q, T* __restrict__ dirs,
                                                   T* __restrict__ lmax, uint8_t* __restrict__ defect,
                                                   double thr, unsigned long long* count) {
    __shared__ unsigned int block_count;
    if (threadIdx.x == 0) block_count = 0;
    __syncthreads();
    const int64_t N = L.N;
    unsigned int mine = 0;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < N;
         s += (int64_t)gridDim.x * blockDim.x) {
        double n[3] = {0.0, 0.0, 0.0}, lam = 0.0;
        const bool sim = (L.mask[s] & M_SIM) != 0;
        if (sim) {
            double v[5];
            for (int c = 0; c < 5; ++c) v[c] = (double)q[c * N + s];
            double Q[3][3];
            full_of(v, Q);
            double p2 = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) p2 += Q[i][j] * Q[i][j];
            if (p2 > 0.0) {
                const double p = sqrt(p2 / 6.0);
                const double det = Q[0][0] * (Q[1][1] * Q[2][2] - Q[1][2] * Q[2][1]) -
                                   Q[0][1] * (Q[1][0] * Q[2][2] - Q[1][2] * Q[2][0]) +
                                   Q[0][2] * (Q[1][0] * Q[2][1] - Q[1][1] * Q[2][0]);
                const double r = fmin(1.0, fmax(-1.0, det / (2.0 * p * p * p)));
                lam = 2.0 * p * cos(acos(r) / 3.0);
                double A[3][3];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) A[i][j] = Q[i][j] - (i == j ? lam : 0.0);
                double best = -1.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = a + 1; b < 3; ++b) {
                        const double c[3] = {A[a][1] * A[b][2] - A[a][2] * A[b][1],
                                             A[a][2] * A[b][0] - A[a][0] * A[b][2],
                                             A[a][0] * A[b][1] - A[a][1] * A[b][0]};
                        const double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
                        if (c2 > best) { best = c2; n[0] = c[0]; n[1] = c[1]; n[2] = c[2]; }
                    }
                if (!(best > 0.0)) {
                    // rank one: a vector normal to the largest row
                    int a = 0;
                    double rb = -1.0;
                    for (int i = 0; i < 3; ++i) {
                        const double r2 = A[i][0] * A[i][0] + A[i][1] * A[i][1] + A[i][2] * A[i][2];
                        if (r2 > rb) { rb = r2; a = i; }
                    }
                    int e = 0;
                    for (int k = 1; k < 3; ++k)
                        if (fabs(A[a][k]) < fabs(A[a][e])) e = k;
                    double u[3] = {0.0, 0.0, 0.0};
                    u[e] = 1.0;
                    n[0] = A[a][1] * u[2] - A[a][2] * u[1];
                    n[1] = A[a][2] * u[0] - A[a][0] * u[2];
                    n[2] = A[a][0] * u[1] - A[a][1] * u[0];
                    best = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
                }
                const double inv = best > 0.0 ? 1.0 / sqrt(best) : 0.0;
                int big = 0;
                for (int k = 1; k < 3; ++k)
                    if (fabs(n[k]) > fabs(n[big])) big = k;
                const double sg = n[big] < 0.0 ? -inv : inv;
                for (int k = 0; k < 3; ++k) n[k] *= sg;
            }
        }
        const bool is_defect = sim && lam < thr;
        mine += is_defect ? 1u : 0u;
        if (dirs)
            for (int k = 0; k < 3; ++k) dirs[k * N + s] = T(n[k]);
        if (lmax) lmax[s] = T(lam);
        if (defect) defect[s] = is_defect ? 1 : 0;
    }
    if (count) {
        atomicAdd(&block_count, mine);
        __syncthreads();
        if (threadIdx.x == 0 && block_count) atomicAdd(count, (unsigned long long)block_count);
    }
}

// ---------------------------------------------------------------------------
// launchers
static int hip_status(hipError_t e) { return e == hipSuccess ? LQ_OK : LQ_EHIP; }

int64_t n_step_blocks(const LatDev& L) { return L.nblocks; }

// Resident blocks per compute unit of the fused FIRE step kernel.
template <typename T, bool L23, bool L4, int W, bool TWO = false>
static int blocks_per_cu() {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_march<T, L23, L4, MODE_FIRE, W, TWO>,
                                                                Tile<T, L23, W>::N, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}
template <typename T>
static int blocks_per_cu_t(bool l23, bool l4, int wide) {
    if (!l23) return wide ? blocks_per_cu<T, false, false, 1>() : blocks_per_cu<T, false, false, 0>();
    if (l4) return wide ? blocks_per_cu<T, true, true, 1>() : blocks_per_cu<T, true, true, 0>();
    return wide ? blocks_per_cu<T, true, false, 1>() : blocks_per_cu<T, true, false, 0>();
}
int step_blocks_per_cu(int prec, bool l23, bool l4, int wide, bool two) {
    if (two && prec == LQ_F64 && l23 && !l4 && wide) return blocks_per_cu<double, true, false, 1, true>();
    return prec == LQ_F64 ? blocks_per_cu_t<double>(l23, l4, wide) : blocks_per_cu_t<float>(l23, l4, wide);
}

int64_t n_energy_blocks(const LatDev& L) {
    int64_t b = (L.N + 255) / 256;
    return b < 2048 ? b : 2048;
}

static int grid_1d(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

template <typename T, int MODE, int W>
static void launch_march(const LatDev& L, bool l23, const Bufs<T>& b, const void* q, void* F, double* partials,
                         FireDev* st, int k, hipStream_t s) {
    const dim3 g((unsigned)n_step_blocks(L));
    if constexpr (sizeof(T) == 8 && W == 1) {
        if (l23 && L.L4 == 0.0 && L.two_waves) {
            k_march<T, true, false, MODE, W, true><<<g, Tile<T, true, W>::N, 0, s>>>(L, b, (const T*)q, (T*)F,
                                                                                 partials, st, k);
            return;
        }
    }
    if (l23 && L.L4 != 0.0)
        k_march<T, true, true, MODE, W><<<g, Tile<T, true, W>::N, 0, s>>>(L, b, (const T*)q, (T*)F, partials, st, k);
    else if (l23)
        k_march<T, true, false, MODE, W><<<g, Tile<T, true, W>::N, 0, s>>>(L, b, (const T*)q, (T*)F, partials, st, k);
    else
        k_march<T, false, false, MODE, W><<<g, Tile<T, false, W>::N, 0, s>>>(L, b, (const T*)q, (T*)F, partials, st, k);
}

template <typename T, int MODE>
static void launch_march_any(const LatDev& L, bool l23, const Bufs<T>& b, const void* q, void* F, double* partials,
                             FireDev* st, int k, hipStream_t s) {
    if (L.wide) launch_march<T, MODE, 1>(L, l23, b, q, F, partials, st, k, s);
    else launch_march<T, MODE, 0>(L, l23, b, q, F, partials, st, k, s);
}

int launch_forces(const LatDev& L, bool l23, int prec, const void* q, void* F, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (prec == LQ_F64) launch_march_any<double, MODE_FORCE>(L, l23, Bufs<double>{}, q, F, nullptr, nullptr, 0, s);
    else launch_march_any<float, MODE_FORCE>(L, l23, Bufs<float>{}, q, F, nullptr, nullptr, 0, s);
    return hip_status(hipGetLastError());
}

template <int MODE>
static void launch_step(const LatDev& L, bool l23, int prec, const void* bufs, double* partials, FireDev* st,
                        int k, hipStream_t s) {
    if (prec == LQ_F64)
        launch_march_any<double, MODE>(L, l23, *(const Bufs<double>*)bufs, nullptr, nullptr, partials, st, k, s);
    else
        launch_march_any<float, MODE>(L, l23, *(const Bufs<float>*)bufs, nullptr, nullptr, partials, st, k, s);
}

// Index of step kernel i (1-based) of a call as the step kernels use it:
// only whether it is the first, and its parity, matter (kept within int).
static int step_index(int64_t i) { return i <= 1 ? (int)i : 2 + (int)(i & 1); }

int launch_fire_steps(const LatDev& L, bool l23, int prec, int method, const void* bufs, double* partials,
                      FireDev* st, int64_t n_steps, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    for (int64_t i = 1; i <= n_steps; ++i) {
        const int k = step_index(i);
        if (method == LQ_METHOD_GD) launch_step<MODE_GD>(L, l23, prec, bufs, partials, st, k, s);
        else if (method == LQ_METHOD_NESTEROV) launch_step<MODE_NAG>(L, l23, prec, bufs, partials, st, k, s);
        else launch_step<MODE_FIRE>(L, l23, prec, bufs, partials, st, k, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return LQ_EHIP;
    }
    // the controller on the last step's reduction, with the step kernel's block size
    const int nt = tile_threads(prec, l23, L.wide), nb = (int)n_step_blocks(L), kl = step_index(n_steps);
    if (nt == 1024) k_dc_control<1024><<<1, 1024, 0, s>>>(st, partials, nb, kl);
    else if (nt == 512) k_dc_control<512><<<1, 512, 0, s>>>(st, partials, nb, kl);
    else if (nt == 256) k_dc_control<256><<<1, 256, 0, s>>>(st, partials, nb, kl);
    else return LQ_EINVAL;
    return hip_status(hipGetLastError());
}

int launch_fire_init_reduce(const LatDev& L, int prec, const void* F, const void* v,
                            double* partials, FireDev* st, void* stream);

int launch_begin(FireDev* st, int64_t n_steps, void* stream) {
    k_begin<<<1, 64, 0, (hipStream_t)stream>>>(st, n_steps);
    return hip_status(hipGetLastError());
}

int launch_finalize(const LatDev& L, int prec, bool with_v, const void* bufs, FireDev* st, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = 5 * L.N;
    if (prec == LQ_F64) k_finalize<double><<<grid_1d(n), 256, 0, s>>>(*(const Bufs<double>*)bufs, n, st, with_v);
    else k_finalize<float><<<grid_1d(n), 256, 0, s>>>(*(const Bufs<float>*)bufs, n, st, with_v);
    if (hipGetLastError() != hipSuccess) return LQ_EHIP;
    k_reset_mix<<<1, 64, 0, s>>>(st);
    return hip_status(hipGetLastError());
}

int launch_lookahead(const LatDev& L, int prec, const void* q, const void* m, double mu, void* y,
                     void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = 5 * L.N;
    if (prec == LQ_F64)
        k_lookahead<double><<<grid_1d(n), 256, 0, s>>>((const double*)q, (const double*)m, mu, (double*)y, n);
    else
        k_lookahead<float><<<grid_1d(n), 256, 0, s>>>((const float*)q, (const float*)m, (float)mu, (float*)y, n);
    return hip_status(hipGetLastError());
}

int launch_directors(const LatDev& L, int prec, const void* q, void* dirs, void* lmax, uint8_t* defect,
                     double thr, unsigned long long* count, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (count) {
        k_fill_zero<<<1, 64, 0, s>>>((uint32_t*)count, 2);
        if (hipGetLastError() != hipSuccess) return LQ_EHIP;
    }
    const int g = grid_1d(L.N);
    if (prec == LQ_F64)
        k_directors<double><<<g, 256, 0, s>>>(L, (const double*)q, (double*)dirs, (double*)lmax, defect, thr, count);
    else
        k_directors<float><<<g, 256, 0, s>>>(L, (const float*)q, (float*)dirs, (float*)lmax, defect, thr, count);
    return hip_status(hipGetLastError());
}

int launch_fill_zero(void* p, int64_t bytes, void* stream) {
    const int64_t w = bytes / 4;
    k_fill_zero<<<grid_1d(w), 256, 0, (hipStream_t)stream>>>((uint32_t*)p, w);
    return hip_status(hipGetLastError());
}

int launch_energy(const LatDev& L, bool l23, int prec, const void* q, double* partials,
                  EnergyOut* out, uint32_t* ticket, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int g = (int)n_energy_blocks(L);
    if (prec == LQ_F64) {
        if (l23) k_energy<double, true><<<g, 256, 0, s>>>(L, (const double*)q, partials, out, ticket);
        else k_energy<double, false><<<g, 256, 0, s>>>(L, (const double*)q, partials, out, ticket);
    } else {
        if (l23) k_energy<float, true><<<g, 256, 0, s>>>(L, (const float*)q, partials, out, ticket);
        else k_energy<float, false><<<g, 256, 0, s>>>(L, (const float*)q, partials, out, ticket);
    }
    return hip_status(hipGetLastError());
}

int launch_uniaxial(const LatDev& L, int prec, const double* dirs, double S, void* q,
                    void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (prec == LQ_F64) k_uniaxial<double><<<grid_1d(L.N), 256, 0, s>>>(L, dirs, S, (double*)q);
    else k_uniaxial<float><<<grid_1d(L.N), 256, 0, s>>>(L, dirs, S, (float*)q);
    return hip_status(hipGetLastError());
}

template <typename T, int W>
static void launch_batch_group(bool l23, const MemberDev* mem, const int* off, int n, int tiles, int k,
                               hipStream_t s) {
    if (n <= 0) return;
    if (l23) k_march_batch<T, true, W><<<tiles, Tile<T, true, W>::N, 0, s>>>(mem, off, n, k);
    else k_march_batch<T, false, W><<<tiles, Tile<T, false, W>::N, 0, s>>>(mem, off, n, k);
}

// The final controller of every member of a group, with the group's block size.
template <typename T, int W>
static void launch_batch_control(bool l23, const MemberDev* mem, int n, int k, hipStream_t s) {
    if (n <= 0) return;
    const int nt = l23 ? Tile<T, true, W>::N : Tile<T, false, W>::N;
    if (nt == 1024) k_batch_dc_control<1024><<<n, 1024, 0, s>>>(mem, k);
    else if (nt == 512) k_batch_dc_control<512><<<n, 512, 0, s>>>(mem, k);
    else k_batch_dc_control<256><<<n, 256, 0, s>>>(mem, k);
}

int launch_batch_steps(int prec, bool l23, const MemberDev* mem, int n_narrow, const int* tile_off,
                       int tiles_narrow, int n_wide, const int* tile_off_wide, int tiles_wide,
                       const int* fin_off, int total_fin, FireDev* gather, int64_t n_steps, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int n_members = n_narrow + n_wide;
    const int nb = (n_members + 63) / 64;
    k_batch_begin<<<nb, 64, 0, s>>>(mem, n_members, n_steps);
    if (hipGetLastError() != hipSuccess) return LQ_EHIP;
    for (int64_t i = 1; i <= n_steps; ++i) {
        const int k = step_index(i);
        if (prec == LQ_F64) {
            launch_batch_group<double, 0>(l23, mem, tile_off, n_narrow, tiles_narrow, k, s);
            launch_batch_group<double, 1>(l23, mem + n_narrow, tile_off_wide, n_wide, tiles_wide, k, s);
        } else {
            launch_batch_group<float, 0>(l23, mem, tile_off, n_narrow, tiles_narrow, k, s);
            launch_batch_group<float, 1>(l23, mem + n_narrow, tile_off_wide, n_wide, tiles_wide, k, s);
        }
        if (hipGetLastError() != hipSuccess) return LQ_EHIP;
    }
    const int kl = step_index(n_steps);
    if (prec == LQ_F64) {
        launch_batch_control<double, 0>(l23, mem, n_narrow, kl, s);
        launch_batch_control<double, 1>(l23, mem + n_narrow, n_wide, kl, s);
    } else {
        launch_batch_control<float, 0>(l23, mem, n_narrow, kl, s);
        launch_batch_control<float, 1>(l23, mem + n_narrow, n_wide, kl, s);
    }
    if (hipGetLastError() != hipSuccess) return LQ_EHIP;
    if (prec == LQ_F64) k_batch_finalize<double><<<total_fin, 256, 0, s>>>(mem, fin_off, n_members);
    else k_batch_finalize<float><<<total_fin, 256, 0, s>>>(mem, fin_off, n_members);
    if (hipGetLastError() != hipSuccess) return LQ_EHIP;
    k_batch_reset_gather<<<nb, 64, 0, s>>>(mem, n_members, gather);
    return hip_status(hipGetLastError());
}

int launch_fire_init_reduce(const LatDev& L, int prec, const void* F, const void* v,
                            double* partials, FireDev* st, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = 5 * L.N;
    const int g = (int)n_energy_blocks(L);
    if (prec == LQ_F64) k_init_reduce<double><<<g, 256, 0, s>>>((const double*)F, (const double*)v, n, partials, st);
    else k_init_reduce<float><<<g, 256, 0, s>>>((const float*)F, (const float*)v, n, partials, st);
    return hip_status(hipGetLastError());
}

}  // namespace lq
