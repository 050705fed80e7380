/*
 * lqfire: lattice Landau-de Gennes force and FIRE relaxation on one MI355X.
 *
 * C ABI of liblqfire.so.  Method: Sussman & Beller, "Fast, scalable, and
 * interactive software for Landau-de Gennes numerical modeling of nematic
 * topological defects" (arXiv:1911.07045).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Lattice: nx * ny * nz sites, site s = x + nx*(y + ny*z), spacing 1.
 *  - Per-site fields (q, v, F) are SoA: component c of site s at [c*N + s],
 *    N = nx*ny*nz, five components (Qxx, Qxy, Qxz, Qyy, Qyz) with
 *    Qzz = -Qxx - Qyy (sec. III.B).  Element type is double for LQ_F64 and
 *    float for LQ_F32.  Field buffers are device memory on the device that was
 *    current at lq_lattice_create, owned by the caller, 5*N elements each,
 *    and must not overlap.
 *  - All device work is enqueued on the stream given at lq_lattice_create.
 *    Calls that return host values (lq_energy, lq_fire_step, lq_minimize,
 *    lq_fire_init) synchronize that stream before returning; lq_compute_forces
 *    and lq_set_uniaxial only enqueue.
 *  - Every call returns LQ_OK (0) or a negative LQ_E* code; no exception or
 *    abort crosses the ABI.  lq_last_error() gives a message.  Errors raised
 *    by the device asynchronously surface as LQ_EHIP at the next call that
 *    synchronizes.
 *  - One lattice handle is used by one host thread at a time.  Handles are
 *    independent of each other.
 */
#ifndef LQFIRE_H
#define LQFIRE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define LQ_OK 0
#define LQ_EINVAL (-1)        /* bad argument: sizes, pointers, NaN/negative parameters */
#define LQ_EUNSUPPORTED (-2)  /* valid in the paper but not built: L6 */
#define LQ_ENOMEM (-3)        /* workspace too small, or a device allocation failed */
#define LQ_EHIP (-4)          /* a HIP runtime call failed */
#define LQ_ENONFINITE (-5)    /* a FIRE reduction produced NaN or Inf */
#define LQ_ESTATE (-6)        /* call order: e.g. lq_fire_step before lq_fire_init */

/* ---- precision of the state ---- */
#define LQ_F64 0 /* q, v, F and all arithmetic in double */
#define LQ_F32 1 /* q, v, F and per-site arithmetic in float; FIRE reductions,
                    controller scalars and the energy sum in double */

typedef struct lq_lattice lq_lattice;

/* Lattice and constants (sec. III.B: everything in units of |A| and dx). */
typedef struct {
    int64_t n[3];        /* nx, ny, nz >= 1; >= 3 on a periodic axis; one field of
                            5 N values must fit in 2^32 bytes (N < 107374182 for
                            LQ_F64, N < 214748364 for LQ_F32) */
    int32_t periodic[3]; /* 1 = periodic axis, 0 = open (neighbours off the edge are absent) */
    int32_t prec;        /* LQ_F64 or LQ_F32 */
    double A, B, C;      /* bulk coefficients, Eq. (fphase); C > 0 */
    double L1, L2, L3;   /* distortion coefficients, Eq. (fdistortionFull) */
    double L4;           /* chiral term (L4/2) eps_lik Q_lj dQ_ij/dx_k of Eq. (fdistortionFull) */
    double L6;           /* must be 0 (LQ_EUNSUPPORTED otherwise) */
} lq_params;

/* Creates a lattice with every site bulk.  stream: a hipStream_t, or NULL for
 * the null stream.  On success *out owns device tables of ~N bytes. */
int lq_lattice_create(const lq_params* p, void* stream, lq_lattice** out);
/* Frees the lattice's tables after its stream's work; a member of a batch
 * leaves the batch first.  NULL is a no-op. */
int lq_lattice_destroy(lq_lattice* lat);

/* S0 of Eq. (S0def) for the lattice's A, B, C (NaN when it has no real value). */
double lq_bulk_S0(const lq_lattice* lat);

/* ---- geometry (sec. III.B site types; sec. II.A.4 anchoring) ---- */
#define LQ_OBJ_WALL 1           /* the lattice plane coordinate[axis] == plane */
#define LQ_OBJ_SPHERE 2         /* sites with |x - center|^2 < radius^2, minimum image on periodic axes */
#define LQ_OBJ_PATTERNED_WALL 3 /* a wall whose preferred director is the in-plane radial unit
                                   vector away from the nearest centre of a square array */
#define LQ_LAW_ND 0             /* W is the Nobili-Durand strength of W tr((Q - Q0)^2) */
#define LQ_LAW_RP 1             /* W is a Rapini-Papoular strength: W >= 0 is used as the
                                   Nobili-Durand strength W / (9 S0^2); W < 0 (degenerate
                                   planar) as the Fournier-Galatola strength |W| / (9 S0^2) */
#define LQ_LAW_FG 2             /* W is the Fournier-Galatola strength of Eq. (planarDegenerate),
                                   W |Qt - P Qt P|^2, Qt = Q + S0/2 I, P = I - nu nu */
#define LQ_DIR_NORMAL 0         /* preferred director = surface normal (homeotropic) */
#define LQ_DIR_FIXED 1          /* preferred director = dir (oriented anchoring) */

typedef struct {
    int32_t kind;      /* LQ_OBJ_* */
    int32_t law;       /* LQ_LAW_* */
    int32_t dir_mode;  /* LQ_DIR_* (ignored by LQ_OBJ_PATTERNED_WALL) */
    int32_t axis;      /* wall axis 0, 1, 2 */
    int64_t plane;     /* wall plane index, 0 <= plane < n[axis] */
    double W;          /* strength >= 0 (a Rapini-Papoular strength may be negative) */
    double center[3];  /* sphere centre (lattice units, any real value) */
    double radius;     /* sphere radius > 0 */
    double dir[3];     /* fixed preferred director (normalized by the library) */
    double pitch[2];   /* patterned wall: centre spacing along the two in-plane axes (ascending order) */
    double offset[2];  /* patterned wall: first centre */
    int32_t count[2];  /* patterned wall: centres per in-plane axis */
} lq_object;

/* One extra anchoring term at a simulated site: the paper's arbitrary
 * per-site anchoring (its custom boundary files).  For a Nobili-Durand term
 * n0 is the preferred director; for a Fournier-Galatola term (LQ_LAW_FG, or
 * LQ_LAW_RP with W < 0) it is the surface normal nu. */
typedef struct {
    int64_t site;
    int32_t law; /* LQ_LAW_* */
    int32_t pad;
    double W;
    double n0[3];
} lq_site_anchor;

/* Replaces the lattice geometry.  Every object marks its interior sites as
 * inside an object (not simulated); object_sites marks extra ones.  A
 * simulated site with a face neighbour inside object a carries one anchoring
 * term of a (so a site touching two objects carries two); recs add more.
 * Nobili-Durand anchoring uses Q0 = 3/2 S0 (n0 n0 - I/3); Fournier-Galatola
 * anchoring uses the surface normal nu of the object (the wall axis, or the
 * unit vector from a sphere's centre) and ignores dir_mode and the patterned
 * wall's radial director (sec. II.A.4).  Host arrays; any may be NULL
 * when its count is 0.  LQ_EINVAL on a bad object, a record at an object site
 * or out of range, S0 not real while anchoring is requested, or more anchored
 * sites than the kernels address (53687091 in FP32, 26843545 in FP64); the
 * previous geometry then stays in place. */
int lq_set_boundaries(lq_lattice* lat, const lq_object* objs, int32_t n_objs,
                      const lq_site_anchor* recs, int64_t n_recs,
                      const int64_t* object_sites, int64_t n_object_sites);

/* Host-only form of the same rasterization (needs no GPU).  Writes the site
 * type of every site to types (N bytes: 0 bulk, 1 boundary, 2 object; may be
 * NULL) and, per anchored site in increasing site order, anch_site[i] and
 * the site's anchoring energy as a quadratic form in its five components,
 * f = 1/2 q^T K q + b^T q + c (every anchoring term is quadratic in Q):
 * anch_data[LQ_ANCH_STRIDE*i ...] = {K00, K01, .., K04, K11, .., K44 (upper
 * triangle, row by row, 15 values), b (5 values), c}; at most cap entries
 * are written (arrays may be NULL when cap is 0).  *n_anchored receives the
 * full count. */
#define LQ_ANCH_STRIDE 21
int lq_rasterize(const lq_params* p, const lq_object* objs, int32_t n_objs,
                 const lq_site_anchor* recs, int64_t n_recs, const int64_t* object_sites,
                 int64_t n_object_sites, uint8_t* types, int64_t* n_anchored,
                 int64_t* anch_site, double* anch_data, int64_t cap);

/* Sets q = 3/2 S (n n - I/3) at simulated sites and 0 inside objects.
 * directors: device, double, [3][N] unit vectors. */
int lq_set_uniaxial(lq_lattice* lat, const double* directors, double S, void* q);

/* ---- forces and energy (sec. III.B) ---- */

/* F = -dE/dq of the discrete energy: bulk Eq. (fphase), distortion
 * Eq. (fdistortionFull) with one-sided differences Eq. (onesidedderivatives)
 * averaged over every allowed choice per axis, anchoring and external
 * fields.  F = 0 inside
 * objects.  q and F: device, 5*N elements. */
int lq_compute_forces(lq_lattice* lat, const void* q, void* F);

/* External fields (sec. II.A.3): each field
 * adds -(chi/3) h_i Q_ij h_j at every simulated site, where h is the field
 * vector and chi the product of the vacuum constant and the anisotropic
 * susceptibility (mu0 dchi for H, eps0 deps for E), in units of |A|.
 * h: host, [n_fields][3]; chi: host, [n_fields].  Replaces the fields set
 * before; n_fields = 0 removes them.  Like lq_set_boundaries it changes the
 * energy, so a bound FIRE state must be initialized again (LQ_ESTATE
 * otherwise).  LQ_EINVAL on non-finite values or n_fields < 0. */
int lq_set_field(lq_lattice* lat, const double* h, const double* chi, int32_t n_fields);

typedef struct {
    double bulk, elastic, anchoring, external, total;
    int64_t n_sim; /* simulated sites */
} lq_energy_terms;

/* Discrete energy of q, summed in double in a fixed order. Synchronizes. */
int lq_energy(lq_lattice* lat, const void* q, lq_energy_terms* out);

/* Director and defect extraction (Eq. Qtensor and the text after it: the
 * director is the eigenvector of Q for its largest eigenvalue, which equals
 * S; the defect display of sec. IV: sites whose largest eigenvalue lies
 * below a threshold).  Per simulated site: dirs (device, [3][N] elements of
 * the lattice's type) receives the unit director with its largest-magnitude
 * component positive (n and -n are one director), lambda_max (device, N
 * elements) the largest eigenvalue, defect (device, N bytes) 1 where
 * lambda_max < threshold.  Sites inside objects and sites with Q = 0 get a
 * zero director and eigenvalue; object sites are never defects.  Any output
 * may be NULL.  n_defects (host, may be NULL) receives the number of defect
 * sites; the call then synchronizes.  Computed in FP64. */
int lq_director_field(lq_lattice* lat, const void* q, void* dirs, void* lambda_max, uint8_t* defect,
                      double threshold, int64_t* n_defects);

/* ---- FIRE (Algorithm 1, after Bitzek et al. 2006) ---- */
typedef struct {
    double dt0, dt_max;  /* initial and largest time step */
    double alpha0;       /* initial steering weight */
    double f_inc, f_dec; /* time-step growth and shrink factors */
    double f_alpha;      /* steering decay factor */
    int64_t n_min;       /* steps with P > 0 before dt grows */
    double force_tol;    /* converged when max |F_i| < force_tol */
    int64_t max_steps;   /* stop after this many steps since lq_fire_init */
} lq_fire_params;

#define LQ_RUNNING 0
#define LQ_CONVERGED 1
#define LQ_MAX_STEPS 2
#define LQ_NONFINITE 3

typedef struct {
    int64_t step;      /* steps taken since lq_fire_init (plus the resumed count) */
    int64_t n_pos;     /* consecutive steps with P > 0 */
    int64_t restarts;  /* steps that took the P <= 0 branch */
    int32_t status;    /* LQ_RUNNING / LQ_CONVERGED / LQ_MAX_STEPS / LQ_NONFINITE */
    int32_t pad;
    double dt, alpha;  /* controller state for the next step */
    double P, normF, normv, maxF; /* F.v, |F|, |v| (before steering) and max |F_i| of the last step */
} lq_fire_report;

/* Bytes of device workspace lq_fire_init needs: a second q, v, F for the
 * ping-pong update, two slots of per-block partial sums (step k writes one
 * while step k + 1 reads the other) and the device FIRE state (two copies and
 * a stop word: each step kernel runs the controller of the step before it). */
int64_t lq_workspace_bytes(const lq_lattice* lat);

/* Binds q, v, F and the workspace to the lattice and starts FIRE: F = F(q),
 * dt = dt0, alpha = alpha0.  resume == NULL: v = 0 and counters at 0.
 * resume != NULL: keeps the caller's v and takes step, n_pos, restarts, dt
 * and alpha from *resume (a report saved earlier), so that a run can be
 * continued bit for bit.  The buffers stay bound until the next
 * lq_fire_init or lq_lattice_destroy. */
int lq_fire_init(lq_lattice* lat, const lq_fire_params* fp, void* q, void* v, void* F,
                 void* workspace, int64_t workspace_bytes, const lq_fire_report* resume);

/* Runs up to n_steps steps of the bound minimizer (FIRE, or the descent
 * bound by lq_descent_init) on the device with no host round trip between
 * steps, stopping early on convergence, max_steps or a non-finite
 * reduction.  On return the bound q, v, F hold the state after the last step
 * (v after steering), and *out the controller.  LQ_ENONFINITE when the run
 * hit a non-finite reduction. */
int lq_fire_step(lq_lattice* lat, int64_t n_steps, lq_fire_report* out);

/* Result of a whole minimization (Algorithm 1 run to its stop test): the
 * final controller, the discrete energy of the final q (sec. III.B) and the
 * per-site force norm |F| / sqrt(N_sim) that the paper plots (Fig. 2). */
typedef struct {
    lq_fire_report fire;     /* status LQ_CONVERGED / LQ_MAX_STEPS / LQ_NONFINITE, steps, max|F_i|, |F| */
    lq_energy_terms energy;  /* energy terms of the final q, as lq_energy gives them */
    double normF_per_site;   /* fire.normF / sqrt(energy.n_sim) */
} lq_min_result;

/* lq_fire_init (fresh) + lq_fire_step until converged or max_steps, then
 * lq_energy of the final q.  out (host, may be NULL) receives the result;
 * when the run stops on a non-finite reduction it returns LQ_ENONFINITE with
 * out->fire filled and the energy terms set to NaN. */
int lq_minimize(lq_lattice* lat, const lq_fire_params* fp, void* q, void* v, void* F,
                void* workspace, int64_t workspace_bytes, lq_min_result* out);

/* ---- allocation-free minimization ----
 * For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lq_minimize
 * without the workspace argument.  The workspace (second q, v, F, partial
 * sums, device FIRE state) lives in a fixed array of
 * LQ_NOALLOC_WORKSPACE_BYTES that the library holds on each GPU it runs on
 * until the process ends; the call allocates nothing (no hipMalloc, hipFree
 * or allocating library routine).  q, v, F are the caller's buffers as for
 * lq_minimize, with the same result and the same trajectory bit for bit.
 * LQ_ENOMEM, before any device work, when lq_workspace_bytes(lat) exceeds
 * LQ_NOALLOC_WORKSPACE_BYTES (64^3 sites fit in FP64, 80^3 in FP32).  Every
 * call on one GPU shares that GPU's array, and it keeps the last call's
 * contents: calls that overlap on one GPU (two host threads, or two streams)
 * race and give undefined results.  The lattice is left unbound on return
 * (lq_fire_step gives LQ_ESTATE), since the next call may reuse the array. */
#define LQ_NOALLOC_WORKSPACE_BYTES ((int64_t)32 << 20)
int lq_minimize_noalloc(lq_lattice* lat, const lq_fire_params* fp, void* q, void* v, void* F,
                        lq_min_result* out);

/* ---- gradient descent and Nesterov's accelerated gradient ----
 * The alternatives to FIRE that sec. III.B names (steepest descent, and
 * Nesterov's momentum method of the GUI).  The paper gives no formulas; the
 * textbook forms are used, with a fixed step dt:
 *   LQ_METHOD_GD:        q <- q + dt F(q)
 *   LQ_METHOD_NESTEROV:  m <- mu m + dt F(q + mu m),  q <- q + m
 * Nesterov keeps m in the v buffer and F at the look-ahead point q + mu m;
 * GD leaves v untouched.  Both run through the same fused kernel as FIRE
 * and are advanced by lq_fire_step, whose report then carries dt, alpha =
 * mu (0 for GD), P = F.m, normv = |m| and n_pos = restarts = 0. */
#define LQ_METHOD_FIRE 0
#define LQ_METHOD_GD 1
#define LQ_METHOD_NESTEROV 2

typedef struct {
    int32_t method;    /* LQ_METHOD_GD or LQ_METHOD_NESTEROV */
    int32_t pad;
    double dt;         /* step, > 0 */
    double momentum;   /* Nesterov mu, 0 <= mu < 1 (ignored by GD) */
    double force_tol;  /* converged when max |F_i| < force_tol */
    int64_t max_steps; /* stop after this many steps since initialization */
} lq_descent_params;

/* Binds q, v, F and the workspace (lq_workspace_bytes) like lq_fire_init and
 * starts the descent: resume == NULL sets v = 0 (Nesterov) and the step
 * count to 0; resume != NULL keeps v and takes the step count from *resume.
 * F = F(q) for GD, F(q + mu v) for Nesterov.  LQ_EINVAL on bad parameters;
 * LQ_ENONFINITE when the initial forces are not finite. */
int lq_descent_init(lq_lattice* lat, const lq_descent_params* dp, void* q, void* v, void* F,
                    void* workspace, int64_t workspace_bytes, const lq_fire_report* resume);

/* lq_descent_init (fresh) + lq_fire_step until converged or max_steps, then
 * lq_energy of the final q; out as for lq_minimize. */
int lq_descent_minimize(lq_lattice* lat, const lq_descent_params* dp, void* q, void* v, void* F,
                        void* workspace, int64_t workspace_bytes, lq_min_result* out);

/* ---- batched FIRE for many small lattices (continuous batching) ----
 * A batch advances all its member lattices by one FIRE step per kernel
 * launch; every member keeps its own controller, partial sums and stop test,
 * so each member follows exactly (bit for bit) the trajectory that
 * lq_fire_step would give it alone.  Members are added and removed between
 * lq_batch_step calls, which is how a serving loop admits and retires
 * requests while others keep running.  All members of a batch share prec
 * and whether L2/L3 are in use, run FIRE (lq_fire_init), and live on the
 * batch's device. */
typedef struct lq_batch lq_batch;

/* capacity: maximum number of members (1 .. 65536).  stream: hipStream_t or
 * NULL; batch steps run on it. */
int lq_batch_create(int32_t capacity, void* stream, lq_batch** out);
int lq_batch_destroy(lq_batch* b);

/* Adds a lattice already bound by lq_fire_init (its stream is synchronized
 * first).  A lattice belongs to at most one batch.  LQ_EINVAL when the batch
 * is full, the lattice is a member of this or another batch, or its prec /
 * L2-L3 use differs from the members'; LQ_ESTATE when it is not bound.
 * Destroying a member lattice removes it from its batch (after the batch's
 * queued work); destroying a batch leaves its lattices intact. */
int lq_batch_add(lq_batch* b, lq_lattice* lat);

/* Removes a member; its buffers keep the state of its last step. */
int lq_batch_remove(lq_batch* b, lq_lattice* lat);

/* Number of members. */
int32_t lq_batch_size(const lq_batch* b);

/* Runs up to n_steps steps for every member (members that have stopped do
 * nothing), then leaves each member's state in its bound q, v, F as
 * lq_fire_step does.  reports: host array of at least lq_batch_size()
 * entries, filled in the order members were added (removals keep the order
 * of the rest).  Synchronizes the batch stream. */
int lq_batch_step(lq_batch* b, int64_t n_steps, lq_fire_report* reports);

/* ---- work plan of the step kernels (host only) ----
 * How the fused step (Algorithm 1 over the whole lattice) is split into
 * blocks for a lattice with the given parameters and objects (as
 * lq_set_boundaries would rasterize them, without records or extra object
 * sites) on a device that keeps `resident` step blocks resident at once
 * (> 0).  A chunk is the X x Y column tile whose first site is (x0, y0), over
 * the planes z0 .. z0 + zc - 1; a block marches one chunk, or two one after
 * the other.  Writes up to cap chunks as 4 int32 each {x0, y0, z0, zc} into
 * chunks, one byte each into bulk (1: every site of the tile, its one-site
 * ring and the planes z0 - 1 and z0 + zc is simulated with all six
 * neighbours) and, if block is not NULL, the index of the block that marches
 * it into block, in launch order (blocks in order, a block's chunks in the
 * order it marches them); *n_chunks receives the full count, *tile_nx and
 * *tile_ny the tile size.  Needs no GPU.  LQ_EINVAL on bad parameters,
 * objects or resident <= 0. */
int lq_step_plan(const lq_params* p, const lq_object* objs, int32_t n_objs, int64_t resident,
                 int32_t* chunks, uint8_t* bulk, int32_t* block, int64_t cap, int64_t* n_chunks,
                 int32_t* tile_nx, int32_t* tile_ny);

/* ---- streaming ceiling (measurement helper) ----
 * A FIRE step (Algorithm 1) reads q, v, F and writes them back: 15 streams in
 * and 15 out per site.  This copies n_streams device buffers of `bytes` each
 * (src[i] -> dst[i], 1..16 streams) with `width` bytes per lane per access
 * (4: one FP32 value per lane, as the FP32 step kernel loads its fields; 8:
 * one FP64 value; 16: whole 16-byte pieces) and the step kernel's
 * non-temporal store policy, so that
 * its time measures what plain streaming of the step's traffic reaches on
 * the device.  Buffers are the caller's device memory, 16-byte aligned, and
 * must not overlap; enqueued on `stream` (a hipStream_t, NULL for the
 * default stream), no synchronization.  LQ_EINVAL on NULL or unaligned
 * pointers, n_streams outside 1..16, width not 4, 8 or 16, or bytes not a
 * positive multiple of width up to 2^31. */
int lq_stream_copy(const void* const* src, void* const* dst, int32_t n_streams, int64_t bytes, int32_t width,
                   void* stream);

/* Message for the last error on lat (or on the calling thread when lat is NULL). */
const char* lq_last_error(const lq_lattice* lat);

#ifdef __cplusplus
}
#endif
#endif /* LQFIRE_H */
