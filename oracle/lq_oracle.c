/*
 * FP64 CPU oracle for the lattice Landau-de Gennes energy, its gradient and
 * the FIRE minimizer (Sussman & Beller, "Fast, scalable, and interactive
 * software for Landau-de Gennes numerical modeling of nematic topological
 * defects", arXiv:1911.07045).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plainly written
 * definition against which the GPU library is checked.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the GPU library.
 *
 * What is computed (paper section III.B, "Lattice discretization and energy
 * minimization", and section II):
 *   - q = (Qxx, Qxy, Qxz, Qyy, Qyz) per site, Qzz = -Qxx - Qyy (sec. III.B);
 *   - bulk density, Eq. (fphase);
 *   - distortion density, Eq. (fdistortionFull) with L6 = 0, built from
 *     the one-sided differences of Eq. (onesidedderivatives) and averaged over
 *     every allowed forward/backward choice per axis (sec. III.B, text after
 *     Eq. onesidedderivatives);
 *   - Nobili-Durand anchoring W tr((Q - Q0)^2) and Fournier-Galatola
 *     degenerate planar anchoring on boundary pairs (sec. II.A.4);
 *   - external fields, linear in Q (sec. II.A.3);
 *   - forces F = -dE/dq by explicit differentiation of the discrete energy
 *     (sec. III.B, the paragraph on explicit differentiation);
 *   - FIRE, Algorithm 1 (after Bitzek et al., PRL 97, 170201 (2006)).
 *
 * Readings of points the paper leaves open are stated where they act.
 *
 * Layout: every per-site field is SoA, component c of site s at [c*N + s],
 * s = x + nx*(y + ny*z).  Site type: 0 bulk, 1 boundary, 2 inside an object.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n[3];          /* nx, ny, nz */
    int32_t periodic[3];   /* 1 = periodic axis */
    double A, B, C;        /* bulk coefficients, Eq. (fphase) */
    double L1, L2, L3;     /* distortion coefficients, Eq. (fdistortionFull) */
    double L4;             /* chiral term of Eq. (fdistortionFull) */
    const uint8_t *type;   /* per site: 0 bulk, 1 boundary, 2 object */
    int64_t n_pairs;       /* anchoring (site, surface) pairs */
    const int64_t *pair_site;
    const double *pair_W;  /* strength used for the pair */
    const double *pair_Q0; /* [n_pairs][5] preferred tensor, q components (Nobili-Durand) */
    const uint8_t *pair_kind; /* 0: Nobili-Durand, 1: Fournier-Galatola (may be NULL: all 0) */
    const double *pair_nu;    /* [n_pairs][3] surface normal (Fournier-Galatola) */
    double S0;                /* bulk order used by Fournier-Galatola, sec. II.A.4 */
    double hfield[9];         /* external-field coupling: f_ext = -sum_ij Q_ij h_ij, sec. II.A.3 */
} ora_problem;

#ifdef _OPENMP
#include <omp.h>
#endif

/* number of threads the parallel loops use */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- Eq. (S0def): the nematic minimum of the uniaxial bulk density ---- */
double ora_S0(double A, double B, double C)
{
    return (-B + sqrt(B * B - 24.0 * A * C)) / (6.0 * C);
}

/* ---- the five independent components -> full symmetric traceless Q ---- */
static void q_to_Q(const double q[5], double Q[3][3])
{
    Q[0][0] = q[0]; Q[0][1] = q[1]; Q[0][2] = q[2];
    Q[1][0] = q[1]; Q[1][1] = q[3]; Q[1][2] = q[4];
    Q[2][0] = q[2]; Q[2][1] = q[4]; Q[2][2] = -q[0] - q[3];
}

/* Chain rule through Q(q): dE/dq_a = sum_ij dE/dQ_ij dQ_ij/dq_a, with the
 * nine entries of the gradient G = dE/dQ taken as independent. */
static void grad_Q_to_q(const double G[3][3], double g[5])
{
    g[0] = G[0][0] - G[2][2];
    g[1] = G[0][1] + G[1][0];
    g[2] = G[0][2] + G[2][0];
    g[3] = G[1][1] - G[2][2];
    g[4] = G[1][2] + G[2][1];
}

static double tr2(const double Q[3][3])
{
    double s = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s += Q[i][j] * Q[j][i];
    return s;
}

static double tr3(const double Q[3][3])
{
    double s = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) s += Q[i][j] * Q[j][k] * Q[k][i];
    return s;
}

/* Eq. (fphase) */
static double f_bulk(const ora_problem *p, const double Q[3][3])
{
    double t2 = tr2(Q);
    return 0.5 * p->A * t2 + p->B / 3.0 * tr3(Q) + 0.25 * p->C * t2 * t2;
}

/* dE/dQ_ab of Eq. (fphase): A Q_ba + B (Q Q)_ba + C tr(Q^2) Q_ba */
static void grad_bulk(const ora_problem *p, const double Q[3][3], double G[3][3])
{
    double t2 = tr2(Q);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double QQ = 0.0;
            for (int k = 0; k < 3; ++k) QQ += Q[b][k] * Q[k][a];
            G[a][b] += p->A * Q[b][a] + p->B * QQ + p->C * t2 * Q[b][a];
        }
}

/* Levi-Civita symbol */
static double eps3(int a, int b, int c)
{
    return (double)((a - b) * (b - c) * (c - a)) / 2.0;
}

/* Eq. (fdistortionFull) with L6 = 0; d[k][i][j] stands for dQ_ij/dx_k and
 * Q is the tensor at the site (it enters the chiral L4 term) */
static double f_dist(const ora_problem *p, const double Q[3][3], double d[3][3][3])
{
    double e1 = 0.0, e2 = 0.0, e3 = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) e1 += d[k][i][j] * d[k][i][j];
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j) s += d[j][i][j];
        e2 += s * s;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) e3 += d[j][i][k] * d[k][i][j];
    double e4 = 0.0;
    for (int l = 0; l < 3; ++l)
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                double e = eps3(l, i, k);
                if (e == 0.0) continue;
                for (int j = 0; j < 3; ++j) e4 += e * Q[l][j] * d[k][i][j];
            }
    return 0.5 * p->L1 * e1 + 0.5 * p->L2 * e2 + 0.5 * p->L3 * e3 + 0.5 * p->L4 * e4;
}

/* derivative of f_dist with respect to d[k][i][j]:
 *   L1 d_k,ij + L2 delta_kj sum_m d_m,im + L3 d_j,ik
 *   + L4/2 sum_l eps_lik Q_lj                                             */
static void grad_dist(const ora_problem *p, const double Q[3][3], double d[3][3][3], double g[3][3][3])
{
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double div = 0.0, chi = 0.0;
                for (int m = 0; m < 3; ++m) div += d[m][i][m];
                for (int l = 0; l < 3; ++l) chi += eps3(l, i, k) * Q[l][j];
                g[k][i][j] = p->L1 * d[k][i][j] + (k == j ? p->L2 * div : 0.0)
                             + p->L3 * d[j][i][k] + 0.5 * p->L4 * chi;
            }
}

/* derivative of f_dist with respect to the site tensor Q_lj (only the L4
 * term depends on it): L4/2 sum_ik eps_lik d_k,ij */
static void grad_dist_site(const ora_problem *p, double d[3][3][3], double h[3][3])
{
    for (int l = 0; l < 3; ++l)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) s += eps3(l, i, k) * d[k][i][j];
            h[l][j] = 0.5 * p->L4 * s;
        }
}

/* ---- lattice helpers ---- */
static int64_t nsites(const ora_problem *p) { return p->n[0] * p->n[1] * p->n[2]; }

/* neighbour of site (c[0],c[1],c[2]) one step along axis k in direction s
 * (+1/-1); returns -1 when it falls off a non-periodic axis */
static int64_t neighbour(const ora_problem *p, const int64_t c[3], int k, int s)
{
    int64_t e[3] = {c[0], c[1], c[2]};
    e[k] += s;
    if (e[k] < 0 || e[k] >= p->n[k]) {
        if (!p->periodic[k]) return -1;
        e[k] = (e[k] + p->n[k]) % p->n[k];
    }
    return e[0] + p->n[0] * (e[1] + p->n[1] * e[2]);
}

static void coords(const ora_problem *p, int64_t s, int64_t c[3])
{
    c[0] = s % p->n[0];
    c[1] = (s / p->n[0]) % p->n[1];
    c[2] = s / (p->n[0] * p->n[1]);
}

static int simulated(const ora_problem *p, int64_t s) { return s >= 0 && p->type[s] != 2; }

static void load_Q(const ora_problem *p, const double *q, int64_t s, double Q[3][3])
{
    int64_t N = nsites(p);
    double v[5];
    for (int a = 0; a < 5; ++a) v[a] = q[a * N + s];
    q_to_Q(v, Q);
}

/* The finite-difference choices allowed at site x along each axis
 * (Eq. onesidedderivatives and the text after it): forward (+1) needs x+e_k
 * simulated, backward (-1) needs x-e_k simulated.  Reading: an axis with no
 * allowed choice contributes the single option "derivative zero" (coded 0). */
typedef struct {
    int n_opt[3];
    int opt[3][2];
    int64_t plus[3], minus[3];
} site_options;

static void options_at(const ora_problem *p, int64_t x, site_options *o)
{
    int64_t c[3];
    coords(p, x, c);
    for (int k = 0; k < 3; ++k) {
        o->plus[k] = neighbour(p, c, k, +1);
        o->minus[k] = neighbour(p, c, k, -1);
        o->n_opt[k] = 0;
        if (simulated(p, o->plus[k])) o->opt[k][o->n_opt[k]++] = +1;
        if (simulated(p, o->minus[k])) o->opt[k][o->n_opt[k]++] = -1;
        if (o->n_opt[k] == 0) o->opt[k][o->n_opt[k]++] = 0;
    }
}

/* one-sided difference along axis k for choice s, Eq. (onesidedderivatives) */
static void difference(const ora_problem *p, const double *q, int64_t x,
                       const site_options *o, int k, int s, double d[3][3])
{
    double Qx[3][3], Qn[3][3];
    if (s == 0) {
        memset(d, 0, 9 * sizeof(double));
        return;
    }
    load_Q(p, q, x, Qx);
    if (s > 0) {
        load_Q(p, q, o->plus[k], Qn);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) d[i][j] = Qn[i][j] - Qx[i][j];
    } else {
        load_Q(p, q, o->minus[k], Qn);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) d[i][j] = Qx[i][j] - Qn[i][j];
    }
}

/* Averaged distortion energy of simulated site x: the mean of f_dist over
 * every combination of allowed choices, one choice per axis. */
static double e_dist_site(const ora_problem *p, const double *q, int64_t x)
{
    site_options o;
    options_at(p, x, &o);
    int ncomb = o.n_opt[0] * o.n_opt[1] * o.n_opt[2];
    double sum = 0.0;
    double d[3][3][3], Qx[3][3];
    load_Q(p, q, x, Qx);
    for (int a = 0; a < o.n_opt[0]; ++a)
        for (int b = 0; b < o.n_opt[1]; ++b)
            for (int c = 0; c < o.n_opt[2]; ++c) {
                int s[3] = {o.opt[0][a], o.opt[1][b], o.opt[2][c]};
                for (int k = 0; k < 3; ++k) difference(p, q, x, &o, k, s[k], d[k]);
                sum += f_dist(p, Qx, d);
            }
    return sum / (double)ncomb;
}

/* Adds d(averaged distortion energy of site x)/dQ(y) to G, by the chain rule
 * through every combination of site x: the difference along axis k depends
 * on Q(y) with coefficient +1 or -1 when y is one of its two end points, and
 * for y = x the chiral term also depends on Q(x) itself. */
static void add_dist_grad_from(const ora_problem *p, const double *q, int64_t x,
                               int64_t y, double G[3][3])
{
    site_options o;
    options_at(p, x, &o);
    int ncomb = o.n_opt[0] * o.n_opt[1] * o.n_opt[2];
    double d[3][3][3], g[3][3][3], Qx[3][3];
    load_Q(p, q, x, Qx);
    for (int a = 0; a < o.n_opt[0]; ++a)
        for (int b = 0; b < o.n_opt[1]; ++b)
            for (int c = 0; c < o.n_opt[2]; ++c) {
                int s[3] = {o.opt[0][a], o.opt[1][b], o.opt[2][c]};
                for (int k = 0; k < 3; ++k) difference(p, q, x, &o, k, s[k], d[k]);
                grad_dist(p, Qx, d, g);
                if (x == y && p->L4 != 0.0) {
                    double h[3][3];
                    grad_dist_site(p, d, h);
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) G[i][j] += h[i][j] / (double)ncomb;
                }
                for (int k = 0; k < 3; ++k) {
                    double coef = 0.0;
                    if (s[k] > 0) {
                        if (o.plus[k] == y) coef += 1.0;
                        if (x == y) coef -= 1.0;
                    } else if (s[k] < 0) {
                        if (x == y) coef += 1.0;
                        if (o.minus[k] == y) coef -= 1.0;
                    }
                    if (coef == 0.0) continue;
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j)
                            G[i][j] += coef * g[k][i][j] / (double)ncomb;
                }
            }
}

/* ---- anchoring of one (site, surface) pair, sec. II.A.4 ----
 * Nobili-Durand:      W tr((Q - Q0)^2)
 * Fournier-Galatola:  W |Qt - P Qt P|^2, Qt = Q + S0/2 I, P = I - nu nu
 * (the projector of Eq. planarDegenerate read as P_ik Qt_kl P_lj). */
static void fg_D(const ora_problem *p, int64_t i, const double Q[3][3], double D[3][3], double P[3][3])
{
    const double *nu = &p->pair_nu[3 * i];
    double Qt[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            P[a][b] = (a == b ? 1.0 : 0.0) - nu[a] * nu[b];
            Qt[a][b] = Q[a][b] + (a == b ? 0.5 * p->S0 : 0.0);
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) s += P[a][k] * Qt[k][l] * P[l][b];
            D[a][b] = Qt[a][b] - s;
        }
}

static int pair_is_fg(const ora_problem *p, int64_t i) { return p->pair_kind && p->pair_kind[i] == 1; }

static double pair_energy(const ora_problem *p, int64_t i, const double Q[3][3])
{
    double t = 0.0;
    if (pair_is_fg(p, i)) {
        double D[3][3], P[3][3];
        fg_D(p, i, Q, D, P);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) t += D[a][b] * D[a][b];
    } else {
        double Q0[3][3];
        q_to_Q(&p->pair_Q0[5 * i], Q0);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) t += (Q[a][b] - Q0[a][b]) * (Q[a][b] - Q0[a][b]);
    }
    return p->pair_W[i] * t;
}

/* adds d(pair energy)/dQ: 2 W (Q - Q0), or 2 W (D - P D P) for Fournier-Galatola */
static void add_pair_grad(const ora_problem *p, int64_t i, const double Q[3][3], double G[3][3])
{
    if (pair_is_fg(p, i)) {
        double D[3][3], P[3][3];
        fg_D(p, i, Q, D, P);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) s += P[a][k] * D[k][l] * P[l][b];
                G[a][b] += 2.0 * p->pair_W[i] * (D[a][b] - s);
            }
    } else {
        double Q0[3][3];
        q_to_Q(&p->pair_Q0[5 * i], Q0);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) G[a][b] += 2.0 * p->pair_W[i] * (Q[a][b] - Q0[a][b]);
    }
}

/* external-field density -sum_ij Q_ij h_ij (linear in Q), sec. II.A.3 */
static double f_ext(const ora_problem *p, const double Q[3][3])
{
    double t = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) t -= Q[a][b] * p->hfield[3 * a + b];
    return t;
}

/* ---- energy: E = sum over simulated sites of (f_bulk + averaged f_dist
 *      + f_ext) + sum over boundary pairs of the anchoring term.
 *      terms[0] bulk, terms[1] distortion, terms[2] anchoring, terms[3]
 *      external field.
 *      Per-plane partial sums are added in plane order, so the result does
 *      not depend on the number of threads. ---- */
double ora_energy(const ora_problem *p, const double *q, double *terms)
{
    int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
    double *pb = (double *)calloc((size_t)nz, sizeof(double));
    double *pd = (double *)calloc((size_t)nz, sizeof(double));
    double *pe = (double *)calloc((size_t)nz, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z) {
        double sb = 0.0, sd = 0.0, se = 0.0;
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t s = x + nx * (y + ny * z);
                if (!simulated(p, s)) continue;
                double Q[3][3];
                load_Q(p, q, s, Q);
                sb += f_bulk(p, Q);
                se += f_ext(p, Q);
                sd += e_dist_site(p, q, s);
            }
        pb[z] = sb;
        pd[z] = sd;
        pe[z] = se;
    }
    double eb = 0.0, ed = 0.0, ea = 0.0, ee = 0.0;
    for (int64_t z = 0; z < nz; ++z) {
        eb += pb[z];
        ed += pd[z];
        ee += pe[z];
    }
    free(pb);
    free(pd);
    free(pe);
    for (int64_t i = 0; i < p->n_pairs; ++i) {
        double Q[3][3];
        load_Q(p, q, p->pair_site[i], Q);
        ea += pair_energy(p, i, Q);
    }
    if (terms) {
        terms[0] = eb;
        terms[1] = ed;
        terms[2] = ea;
        terms[3] = ee;
    }
    return eb + ed + ea + ee;
}

/* ---- forces F = -dE/dq.  Each site y gathers the derivative of every
 *      energy term that contains Q(y): its own bulk term, the averaged
 *      distortion terms of itself and of its six face neighbours, and its
 *      anchoring pairs.  Sites inside objects carry no degrees of freedom and
 *      get F = 0. ---- */
void ora_forces(const ora_problem *p, const double *q, double *F)
{
    int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
    int64_t N = nsites(p);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t yy = 0; yy < ny; ++yy)
            for (int64_t xx = 0; xx < nx; ++xx) {
                int64_t y = xx + nx * (yy + ny * z);
                double G[3][3] = {{0}};
                double g[5] = {0};
                if (simulated(p, y)) {
                    double Q[3][3];
                    load_Q(p, q, y, Q);
                    grad_bulk(p, Q, G);
                    for (int a = 0; a < 9; ++a) G[a / 3][a % 3] -= p->hfield[a];
                    add_dist_grad_from(p, q, y, y, G);
                    int64_t c[3] = {xx, yy, z};
                    for (int k = 0; k < 3; ++k)
                        for (int s = -1; s <= 1; s += 2) {
                            int64_t x = neighbour(p, c, k, s);
                            if (simulated(p, x)) add_dist_grad_from(p, q, x, y, G);
                        }
                    grad_Q_to_q(G, g);
                }
                for (int a = 0; a < 5; ++a) F[a * N + y] = -g[a];
            }
    /* anchoring, serial over pairs */
    for (int64_t i = 0; i < p->n_pairs; ++i) {
        int64_t s = p->pair_site[i];
        double Q[3][3], Ga[3][3] = {{0}}, g[5];
        load_Q(p, q, s, Q);
        add_pair_grad(p, i, Q, Ga);
        grad_Q_to_q(Ga, g);
        for (int a = 0; a < 5; ++a) F[a * N + s] -= g[a];
    }
}

/* ---- FIRE, Algorithm 1, over a flat vector of n_dof unknowns ----
 * Readings (the paper names the steps, Bitzek et al. 2006 give the
 * constants): alpha follows Bitzek's convention, i.e. it is the steering
 * weight that starts at alpha0 and is multiplied by f_alpha once P has been
 * positive for more than N_min steps; the counter is incremented before that
 * test; P <= 0 takes the restart branch; q is not rolled back on a restart;
 * there is no floor on dt; the stop test uses the largest force component. */
typedef struct {
    double dt0, dt_max, alpha0, f_inc, f_dec, f_alpha;
    int64_t n_min;
    double force_tol;   /* stop when max |F_i| < force_tol */
    int64_t max_steps;  /* stop when step == max_steps */
} ora_fire_params;

enum { ORA_RUNNING = 0, ORA_CONVERGED = 1, ORA_MAX_STEPS = 2, ORA_NONFINITE = 3 };

typedef struct {
    double dt, alpha;
    int64_t n_pos, step, restarts;
    int32_t status;
    int32_t pad;
    double P, normF, normv, maxF;  /* values measured at the last step */
} ora_fire_state;

typedef void (*ora_force_fn)(void *ctx, const double *x, double *F);

static double max_abs(int64_t n, const double *F)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double a = fabs(F[i]);
        if (a > m || a != a) m = a;
    }
    return m;
}

/* v = 0 unless keep_v; F = force(x); fresh controller */
void ora_fire_init(const ora_fire_params *fp, ora_fire_state *st, int64_t n, const double *x,
                   double *v, double *F, ora_force_fn force, void *ctx, int keep_v)
{
    if (!keep_v) memset(v, 0, (size_t)n * sizeof(double));
    force(ctx, x, F);
    st->dt = fp->dt0;
    st->alpha = fp->alpha0;
    st->n_pos = 0;
    st->step = 0;
    st->restarts = 0;
    st->P = 0.0;
    st->normF = 0.0;
    st->normv = 0.0;
    st->maxF = max_abs(n, F);
    st->status = ORA_RUNNING;
    if (!(st->maxF == st->maxF)) st->status = ORA_NONFINITE;
    else if (st->maxF < fp->force_tol) st->status = ORA_CONVERGED;
    else if (st->step >= fp->max_steps) st->status = ORA_MAX_STEPS;
}

/* Runs up to n_steps iterations of Algorithm 1.  trace (optional) receives,
 * per step, {P, |F|, |v|, max|F|, dt, alpha} as they stand after the step.
 * Returns the number of steps taken. */
int64_t ora_fire_steps(const ora_fire_params *fp, ora_fire_state *st, int64_t n, double *x,
                       double *v, double *F, ora_force_fn force, void *ctx, int64_t n_steps,
                       double *trace)
{
    int64_t taken = 0;
    while (taken < n_steps && st->status == ORA_RUNNING) {
        double dt = st->dt;
        /* velocity Verlet step */
        for (int64_t i = 0; i < n; ++i) v[i] += 0.5 * dt * F[i];
        for (int64_t i = 0; i < n; ++i) x[i] += dt * v[i];
        force(ctx, x, F);
        for (int64_t i = 0; i < n; ++i) v[i] += 0.5 * dt * F[i];
        st->step += 1;
        taken += 1;
        /* power and norms */
        double P = 0.0, f2 = 0.0, v2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            P += F[i] * v[i];
            f2 += F[i] * F[i];
            v2 += v[i] * v[i];
        }
        double nF = sqrt(f2), nv = sqrt(v2);
        st->P = P;
        st->normF = nF;
        st->normv = nv;
        st->maxF = max_abs(n, F);
        if (!(P == P) || !(f2 == f2) || !(v2 == v2) || isinf(P) || isinf(f2) || isinf(v2)) {
            st->status = ORA_NONFINITE;
            break;
        }
        if (P > 0.0) {
            /* steer the velocity toward the force */
            double a = st->alpha;
            for (int64_t i = 0; i < n; ++i) v[i] = (1.0 - a) * v[i] + a * nv * F[i] / nF;
            st->n_pos += 1;
            if (st->n_pos > fp->n_min) {
                st->dt = fmin(st->dt * fp->f_inc, fp->dt_max);
                st->alpha = st->alpha * fp->f_alpha;
            }
        } else {
            /* restart: freeze, shrink the step, reset the steering */
            memset(v, 0, (size_t)n * sizeof(double));
            st->dt = st->dt * fp->f_dec;
            st->alpha = fp->alpha0;
            st->n_pos = 0;
            st->restarts += 1;
        }
        if (trace) {
            double *t = trace + 6 * (taken - 1);
            t[0] = P; t[1] = nF; t[2] = nv; t[3] = st->maxF; t[4] = st->dt; t[5] = st->alpha;
        }
        if (st->maxF < fp->force_tol) st->status = ORA_CONVERGED;
        else if (st->step >= fp->max_steps) st->status = ORA_MAX_STEPS;
    }
    return taken;
}

/* ---- gradient descent and Nesterov's accelerated gradient (sec. III.C
 * names both as alternatives to FIRE; the paper gives no formulas, so the
 * textbook forms are taken):
 *   GD:        q <- q + dt F(q)                     (steepest descent, i.e.
 *              overdamped dynamics at zero temperature)
 *   Nesterov:  m <- mu m + dt F(q + mu m);  q <- q + m
 * The force is always kept at the point where it was last evaluated:
 * F(q) for GD, F(y) with y = q + mu m for Nesterov, and the stop test uses
 * the largest component of that force.  Reported per step: P = F.m,
 * |F|, |m|, max|F| (m stays untouched by GD). ---- */
enum { ORA_GD = 1, ORA_NESTEROV = 2 };

typedef struct {
    int32_t method;     /* ORA_GD or ORA_NESTEROV */
    int32_t pad;
    double dt, momentum;
    double force_tol;
    int64_t max_steps;
} ora_descent_params;

static void lookahead(int64_t n, const double *x, const double *m, double mu, double *y)
{
    for (int64_t i = 0; i < n; ++i) y[i] = x[i] + mu * m[i];
}

static void measure(const ora_descent_params *dp, ora_fire_state *st, int64_t n, const double *m,
                    const double *F)
{
    double P = 0.0, f2 = 0.0, m2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        P += F[i] * m[i];
        f2 += F[i] * F[i];
        m2 += m[i] * m[i];
    }
    st->P = P;
    st->normF = sqrt(f2);
    st->normv = sqrt(m2);
    st->maxF = max_abs(n, F);
    if (!isfinite(P) || !isfinite(f2) || !isfinite(m2) || !(st->maxF == st->maxF)) st->status = ORA_NONFINITE;
    else if (st->maxF < dp->force_tol) st->status = ORA_CONVERGED;
    else if (st->step >= dp->max_steps) st->status = ORA_MAX_STEPS;
}

/* m = 0 unless keep_m; F = force at q (GD) or at q + mu m (Nesterov) */
void ora_descent_init(const ora_descent_params *dp, ora_fire_state *st, int64_t n, const double *x,
                      double *m, double *F, ora_force_fn force, void *ctx, int keep_m)
{
    if (!keep_m) memset(m, 0, (size_t)n * sizeof(double));
    if (dp->method == ORA_NESTEROV) {
        double *y = (double *)malloc((size_t)n * sizeof(double));
        lookahead(n, x, m, dp->momentum, y);
        force(ctx, y, F);
        free(y);
    } else {
        force(ctx, x, F);
    }
    memset(st, 0, sizeof(*st));
    st->dt = dp->dt;
    st->alpha = dp->method == ORA_NESTEROV ? dp->momentum : 0.0;
    st->status = ORA_RUNNING;
    measure(dp, st, n, m, F);
}

int64_t ora_descent_steps(const ora_descent_params *dp, ora_fire_state *st, int64_t n, double *x,
                          double *m, double *F, ora_force_fn force, void *ctx, int64_t n_steps,
                          double *trace)
{
    int64_t taken = 0;
    double *y = dp->method == ORA_NESTEROV ? (double *)malloc((size_t)n * sizeof(double)) : NULL;
    while (taken < n_steps && st->status == ORA_RUNNING) {
        if (dp->method == ORA_NESTEROV) {
            for (int64_t i = 0; i < n; ++i) m[i] = dp->momentum * m[i] + dp->dt * F[i];
            for (int64_t i = 0; i < n; ++i) x[i] += m[i];
            lookahead(n, x, m, dp->momentum, y);
            force(ctx, y, F);
        } else {
            for (int64_t i = 0; i < n; ++i) x[i] += dp->dt * F[i];
            force(ctx, x, F);
        }
        st->step += 1;
        taken += 1;
        measure(dp, st, n, m, F);
        if (trace) {
            double *t = trace + 6 * (taken - 1);
            t[0] = st->P; t[1] = st->normF; t[2] = st->normv; t[3] = st->maxF; t[4] = st->dt;
            t[5] = st->alpha;
        }
    }
    free(y);
    return taken;
}

/* lattice force as an ora_force_fn */
static void lattice_force(void *ctx, const double *x, double *F)
{
    ora_forces((const ora_problem *)ctx, x, F);
}

void ora_fire_init_lattice(const ora_problem *p, const ora_fire_params *fp, ora_fire_state *st,
                           const double *q, double *v, double *F, int keep_v)
{
    ora_fire_init(fp, st, 5 * nsites(p), q, v, F, lattice_force, (void *)p, keep_v);
}

int64_t ora_fire_steps_lattice(const ora_problem *p, const ora_fire_params *fp, ora_fire_state *st,
                               double *q, double *v, double *F, int64_t n_steps, double *trace)
{
    return ora_fire_steps(fp, st, 5 * nsites(p), q, v, F, lattice_force, (void *)p, n_steps, trace);
}

void ora_descent_init_lattice(const ora_problem *p, const ora_descent_params *dp, ora_fire_state *st,
                              const double *q, double *m, double *F, int keep_m)
{
    ora_descent_init(dp, st, 5 * nsites(p), q, m, F, lattice_force, (void *)p, keep_m);
}

int64_t ora_descent_steps_lattice(const ora_problem *p, const ora_descent_params *dp, ora_fire_state *st,
                                  double *q, double *m, double *F, int64_t n_steps, double *trace)
{
    return ora_descent_steps(dp, st, 5 * nsites(p), q, m, F, lattice_force, (void *)p, n_steps, trace);
}

/* ---- force at a list of sites only (for sampled checks on lattices too
 *      large for a full pass); out is [n_sites][5]; anchoring included ---- */
void ora_forces_at(const ora_problem *p, const double *q, int64_t n_sites, const int64_t *sites,
                   double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_sites; ++i) {
        int64_t y = sites[i];
        double G[3][3] = {{0}};
        double g[5] = {0};
        if (simulated(p, y)) {
            double Q[3][3];
            int64_t c[3];
            coords(p, y, c);
            load_Q(p, q, y, Q);
            grad_bulk(p, Q, G);
            for (int a = 0; a < 9; ++a) G[a / 3][a % 3] -= p->hfield[a];
            add_dist_grad_from(p, q, y, y, G);
            for (int k = 0; k < 3; ++k)
                for (int s = -1; s <= 1; s += 2) {
                    int64_t x = neighbour(p, c, k, s);
                    if (simulated(p, x)) add_dist_grad_from(p, q, x, y, G);
                }
            for (int64_t j = 0; j < p->n_pairs; ++j)
                if (p->pair_site[j] == y) add_pair_grad(p, j, Q, G);
            grad_Q_to_q(G, g);
        }
        for (int a = 0; a < 5; ++a) out[5 * i + a] = -g[a];
    }
}
