/*
 * biot_oracle.c -- plain FP64 CPU oracle of the semi-implicit lattice Boltzmann
 * scheme for Biot's consolidation model (Lunowa & Wohlmuth, arXiv:2409.11382).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the HIP path is checked against.  It shares no code, header, table or
 * constant with the HIP library; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * Everything is computed in lattice units (lattice spacing and time step 1,
 * c_s^2 = 1/3).  The dimensional inputs are converted as follows (the reading of
 * the paper's mixed units; Sec. 2.2 and the end of Sec. 3.4):
 *   lambda' = c0 lambda, mu' = c0 mu, kappa' = kappa / c0,
 *   elastic force per collision      F = h^2 c0 f - alpha h grad_lat p',
 *   traction term                    h * (c0 t),
 *   pressure                         p' = c0 p,
 *   flow source per step             s_lat = dt s - (alpha/h) * (change of D),
 *   D = lattice divergence of eta    (eq. LBM:divergence),
 *   lattice diffusivity              k = kappa' dt / h^2, omega_f = 1/(3k + 1/2)
 *                                    (eq. pressure:rate).
 * Layout: array-of-structures, cell (x, y) at index y*nx + x.
 *
 * Pins: every function is checked by tests/test_oracle_pins.py and
 * tests/test_oracle_cycles.py against closed forms, exact invariants,
 * brute-force solves, convergence to series solutions or values the paper
 * states.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- tables */
/* D2Q9, Table 1: linear index 0..8 and weights. */
static const int C9X[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int C9Y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* D2Q8, Fig. 1 (Miller indices): 10, 01, -10, 0-1, 11, -11, -1-1, 1-1.
 * Weights: the non-rest D2Q9 weights, which the Dirichlet rule eq. BC:elasticity
 * relies on. */
static const int C8X[8] = {1, 0, -1, 0, 1, -1, -1, 1};
static const int C8Y[8] = {0, 1, 0, -1, 1, 1, -1, -1};
static const double W8[8] = {1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* Table 3 as printed: rows are g_ij in the order above, columns in the printed
 * order (01, 10, 11, s, d, 12, 21, 22).  The first two column headers are
 * swapped in print: the first column multiplies m10 and the second m01 (only
 * that reading inverts eqs. moments/moments:stress). */
static const double TAB3[8][8] = {
    { 0.5,  0.0,  0.0,  0.25,  0.25, -0.5,  0.0, -0.5},
    { 0.0,  0.5,  0.0,  0.25, -0.25,  0.0, -0.5, -0.5},
    {-0.5,  0.0,  0.0,  0.25,  0.25,  0.5,  0.0, -0.5},
    { 0.0, -0.5,  0.0,  0.25, -0.25,  0.0,  0.5, -0.5},
    { 0.0,  0.0,  0.25, 0.0,   0.0,   0.25, 0.25, 0.25},
    { 0.0,  0.0, -0.25, 0.0,   0.0,  -0.25, 0.25, 0.25},
    { 0.0,  0.0,  0.25, 0.0,   0.0,  -0.25, -0.25, 0.25},
    { 0.0,  0.0, -0.25, 0.0,   0.0,   0.25, -0.25, 0.25},
};
/* column meaning under the corrected reading */
enum { T_M10 = 0, T_M01 = 1, T_M11 = 2, T_MS = 3, T_MD = 4, T_M12 = 5, T_M21 = 6, T_M22 = 7 };

enum { LEFT = 0, RIGHT = 1, BOTTOM = 2, TOP = 3 };
enum { FL_PERIODIC = 0, FL_DIRICHLET = 1, FL_NOFLOW = 2, FL_SYMMETRY = 3 };
enum { EL_PERIODIC = 0, EL_DIRICHLET = 1, EL_TRACTION = 2, EL_SYMMETRY = 3 };

enum { OR_OK = 0, OR_ERR_ARG = -1, OR_ERR_DIVERGED = -4, OR_ERR_STATE = -6, OR_ERR_NOMEM = -7 };

/* ---------------------------------------------------------------- API types */
typedef struct {
    int32_t nx, ny;
    double dx, dt, lambda, mu, c0, alpha;
    const double *kappa;          /* N values or NULL */
    double kappa_uniform;
    double r;
    int32_t levels, K;
    double gamma;
    int32_t ne_fixed;
    double ne_tol;
    int32_t ne_max;
    int32_t el_type[4];
    const int8_t *flow_type[4];   /* per boundary cell */
    const double *el_value[4];    /* 2 per boundary cell */
    const double *p_value[4];     /* 1 per boundary cell */
    int32_t pressure_gradient;    /* 0: eq. pressure:gradient, 1: eq. pressure:gradient:alternative */
    int32_t cycle;                /* 0: V-cycle (Algorithm 4), 1: W-cycle, 2: F-cycle,
                                     3: full multigrid (first cycle of a step), then V */
    int32_t fstar_literal;        /* 1: self-dependence constant alpha^2/2 as printed in
                                     eq. MG:selfdependence, for every r; 0: r alpha^2/2 */
    int32_t coarse_sweeps;        /* smoothing steps on the coarsest level of a multigrid
                                     hierarchy (levels >= 2); 0: the 2K of Algorithm 4 */
    int32_t lag;                  /* Algorithm 1 only (one level, gamma = 1): the implicit
                                     source uses the divergence of the previous pseudo-time
                                     step (eq. source:implicit) instead of the current one */
} or_problem;

typedef struct {
    int nx, ny, n;
    /* boundary data of this level: zero on every coarse level (homogeneous
     * versions of the fine-level conditions, Sec. 3.5) */
    double *el_val[4];   /* 2 per boundary cell, already in lattice units */
    /* work arrays used by the multigrid recursion at this level */
    double *g, *r, *u, *F, *D, *gs, *S, *tmp;
} level_t;

typedef struct {
    or_problem pb;
    int nx, ny, n, L, K;
    double h, dt, gamma, r, alpha, c0;
    double lam, mu;          /* c0-scaled */
    double om_s, om_d, b_s, b_d, beta22, cstar;
    double *om_f;            /* per cell */
    int el_type[4];
    int8_t *flow_type[4];
    double *p_bc[4];         /* c0-scaled pressure data */
    level_t *lv;             /* lv[1..L], lv[L] finest */
    /* state */
    double *f, *g, *D1, *D2;
    double *Ft;              /* explicit force of the current step */
    double *fbody;           /* c0 h^2 f (lattice), 2 per cell */
    double *src;             /* dt * s, 1 per cell */
    int step;
    int status;
    /* outputs of the last completed step */
    double *eta, *p, *sig;
    /* statistics */
    int *ne_hist; double *ratio_hist; int hist_cap;
    const int *ne_sched; int ne_sched_len;
    int threads;
    long coarsest_visits;    /* coarsest-level solves so far (cycle-shape pins) */
    double *Dlag;            /* Algorithm 1 with the lag: divergence of the previous
                                pseudo-time step's iterate */
} or_state;

/* ---------------------------------------------------------------- helpers */
static int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }
static int wrapi(int i, int n) { i %= n; return i < 0 ? i + n : i; }
static int opp8(int q) { for (int k = 0; k < 8; ++k) if (C8X[k] == -C8X[q] && C8Y[k] == -C8Y[q]) return k; return -1; }
static int opp9(int i) { for (int k = 0; k < 9; ++k) if (C9X[k] == -C9X[i] && C9Y[k] == -C9Y[i]) return k; return -1; }
static int find8(int cx, int cy) { for (int k = 0; k < 8; ++k) if (C8X[k] == cx && C8Y[k] == cy) return k; return -1; }
static int find9(int cx, int cy) { for (int k = 0; k < 9; ++k) if (C9X[k] == cx && C9Y[k] == cy) return k; return -1; }

static int side_periodic(const or_state *o, int side) { return o->el_type[side] == EL_PERIODIC; }

/* raw moment m_ab = sum_ij i^a j^b g_ij (eq. moments) */
static double raw_moment(const double g[8], int a, int b)
{
    double m = 0.0;
    for (int q = 0; q < 8; ++q) m += (double)(ipow(C8X[q], a) * ipow(C8Y[q], b)) * g[q];
    return m;
}

/* m_s of eq. moments:stress */
static double moment_s(const double g[8]) { return raw_moment(g, 2, 0) + raw_moment(g, 0, 2); }

/* lattice divergence of eta from the populations, eq. LBM:divergence with the
 * bared moment of eq. moments:bared */
static double divergence_of(const or_state *o, const double g[8])
{
    return -(o->b_s * moment_s(g)) / (2.0 * (o->lam + o->mu));
}

/* ghost index for the central gradient: periodic wrap, otherwise even
 * reflection across the wall (ghost -k equals cell k-1) */
static int ghost_index(int i, int n, int periodic)
{
    if (i >= 0 && i < n) return i;
    if (periodic) return wrapi(i, n);
    if (i < 0) return -i - 1;
    return 2 * n - 1 - i;
}

/* central difference gradient, eq. pressure:gradient:alternative in lattice
 * units: grad q(x) = sum_i w_i c_i q(x + c_i) / c_s^2 */
static void grad_central(const or_state *o, int nx, int ny, const double *q, double *out /*2 per cell*/)
{
    int px = side_periodic(o, LEFT), py = side_periodic(o, BOTTOM);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double gx = 0.0, gy = 0.0;
            for (int i = 1; i < 9; ++i) {
                int xs = ghost_index(x + C9X[i], nx, px);
                int ys = ghost_index(y + C9Y[i], ny, py);
                double v = q[ys * nx + xs];
                gx += W9[i] * C9X[i] * v * 3.0;
                gy += W9[i] * C9Y[i] * v * 3.0;
            }
            out[2 * (y * nx + x) + 0] = gx;
            out[2 * (y * nx + x) + 1] = gy;
        }
}

/* self-dependence force F_*(g) = C* grad^c D(g) (eq. MG:selfdependence) with
 * C* = r alpha^2 / 2, the implicit share of the centred source of eq.
 * source:implicit, or the printed alpha^2 / 2 for every r (fstar_literal) */
static void self_force(const or_state *o, const level_t *lv, const double *g, double *D, double *Fs)
{
#pragma omp parallel for schedule(static)
    for (int c = 0; c < lv->n; ++c) D[c] = divergence_of(o, g + 8 * c);
    grad_central(o, lv->nx, lv->ny, D, Fs);
    for (int c = 0; c < 2 * lv->n; ++c) Fs[c] *= o->cstar;
}

/* ------------------------------------------------------- elastic collision */
/* Algorithm 2, collision part: moments, half force, equilibrium, half force,
 * relaxation (Table 2), back-transformation (Table 3 with eq. moments:collision:22). */
static void elastic_collide(const or_state *o, const double u[8], const double F[2], double out[8])
{
    /* moments */
    double m10 = raw_moment(u, 1, 0), m01 = raw_moment(u, 0, 1), m11 = raw_moment(u, 1, 1);
    double m20 = raw_moment(u, 2, 0), m02 = raw_moment(u, 0, 2);
    double ms = m20 + m02, md = m20 - m02;
    /* first half force (eq. moments:halfForce) */
    double mb10 = m10 + 0.5 * F[0], mb01 = m01 + 0.5 * F[1];
    /* equilibrium moments, Table 2 */
    double eq_s = 0.0, eq_d = 0.0, eq_11 = 0.0, eq_12 = mb10 / 3.0, eq_21 = mb01 / 3.0;
    /* second half force */
    double st10 = mb10 + 0.5 * F[0], st01 = mb01 + 0.5 * F[1];
    /* relaxation (eq. moments:collision, rates of Table 2; omega_12 = omega_21 = 1) */
    double m12 = raw_moment(u, 1, 2), m21 = raw_moment(u, 2, 1);
    double sts = ms - o->om_s * (ms - eq_s);
    double std_ = md - o->om_d * (md - eq_d);
    double st11 = m11 - o->om_d * (m11 - eq_11);
    double st12 = m12 - 1.0 * (m12 - eq_12);
    double st21 = m21 - 1.0 * (m21 - eq_21);
    /* eq. moments:collision:22 (m_f relaxed with rate 1 to zero) */
    double st22 = -o->beta22 * ms;
    double mstar[8];
    mstar[T_M10] = st10; mstar[T_M01] = st01; mstar[T_M11] = st11; mstar[T_MS] = sts;
    mstar[T_MD] = std_;  mstar[T_M12] = st12; mstar[T_M21] = st21; mstar[T_M22] = st22;
    /* back-transformation, eq. moments:inverse */
    for (int q = 0; q < 8; ++q) {
        double v = 0.0;
        for (int k = 0; k < 8; ++k) v += TAB3[q][k] * mstar[k];
        out[q] = v;
    }
}

/* ------------------------------------------------------ elastic boundaries */
/* value of the boundary data of `side` at the midpoint of the link that leaves
 * the boundary cell (x, y) in direction (ox, oy) (halfway point of the link).
 * Data are given at the face centres of the boundary cells.  Axis links take the
 * cell's face value; a diagonal link ends at a corner point of the face, whose
 * value is the mean of the two face values beside it.  At the end of a side the
 * second value comes from the perpendicular side's condition: periodic wrap,
 * the mirror image for a symmetry wall (for vector data the component normal to
 * the mirror changes sign), otherwise linear extrapolation along the side. */
static void link_data(const or_state *o, int nx, int ny, const double *vals, int ncomp,
                      int side, int x, int y, int ox, int oy, double *out)
{
    int idx, tn, n, perp, mirror_comp;
    if (side == LEFT || side == RIGHT) {
        idx = y; tn = y + oy; n = ny; perp = (tn < 0) ? BOTTOM : TOP; mirror_comp = 1;
    } else {
        idx = x; tn = x + ox; n = nx; perp = (tn < 0) ? LEFT : RIGHT; mirror_comp = 0;
    }
    for (int k = 0; k < ncomp; ++k) out[k] = vals[ncomp * idx + k];
    if (ox == 0 || oy == 0) return;
    double other[2];
    /* kind of the perpendicular wall at this end of the side: the elastic type
     * for displacement/traction data, the corner cell's flow type for p_D */
    int pk;
    if (ncomp == 2) pk = o->el_type[perp];
    else {
        int cx = (side == LEFT || side == RIGHT) ? x : (perp == LEFT ? 0 : nx - 1);
        int cy = (side == LEFT || side == RIGHT) ? (perp == BOTTOM ? 0 : ny - 1) : y;
        int ft = o->flow_type[perp][(perp == LEFT || perp == RIGHT) ? cy : cx];
        pk = (ft == FL_PERIODIC) ? EL_PERIODIC : (ft == FL_SYMMETRY) ? EL_SYMMETRY : EL_DIRICHLET;
    }
    if (tn >= 0 && tn < n) {
        for (int k = 0; k < ncomp; ++k) other[k] = vals[ncomp * tn + k];
    } else if (pk == EL_PERIODIC) {
        tn = wrapi(tn, n);
        for (int k = 0; k < ncomp; ++k) other[k] = vals[ncomp * tn + k];
    } else if (pk == EL_SYMMETRY) {
        for (int k = 0; k < ncomp; ++k)
            other[k] = (ncomp == 2 && k == mirror_comp) ? -out[k] : out[k];
    } else {
        int in = 2 * idx - tn;   /* the neighbour on the other side */
        if (in < 0 || in >= n) return;
        for (int k = 0; k < ncomp; ++k) other[k] = 2.0 * out[k] - vals[ncomp * in + k];
    }
    for (int k = 0; k < ncomp; ++k) out[k] = 0.5 * (out[k] + other[k]);
}

/* traction correction for the incoming direction q at a wall with outward
 * normal n: the stress implied by the traction t = sigma n is sigma_nn = n.t and
 * sigma_12 = (shear of t); varsigma = -sigma_nn on the axis link and
 * -(1/2) c_x c_y sigma_12 on diagonal links (eq. BC:traction and the left-wall
 * formulas after it, carried over to the other walls). */
static double traction_term(int side, int q, const double t[2])
{
    int nxn = (side == LEFT) ? -1 : (side == RIGHT) ? 1 : 0;
    int nyn = (side == BOTTOM) ? -1 : (side == TOP) ? 1 : 0;
    double sig_nn = nxn * t[0] + nyn * t[1];
    double sig_12 = (nxn != 0) ? nxn * t[1] : nyn * t[0];
    if (C8X[q] != 0 && C8Y[q] != 0) return -0.5 * C8X[q] * C8Y[q] * sig_12;
    return -sig_nn;
}

/* population q arriving at (x, y) after streaming, eq. streaming with the
 * boundary rules of Sec. 3.6. gs holds post-collision populations. */
static double elastic_incoming(const or_state *o, const level_t *lv, const double *gs, int x, int y, int q)
{
    int nx = lv->nx, ny = lv->ny;
    int sx = x - C8X[q], sy = y - C8Y[q];
    int outx = (sx < 0 || sx >= nx), outy = (sy < 0 || sy >= ny);
    if (outx && side_periodic(o, LEFT)) { sx = wrapi(sx, nx); outx = 0; }
    if (outy && side_periodic(o, BOTTOM)) { sy = wrapi(sy, ny); outy = 0; }
    if (!outx && !outy) return gs[8 * (sy * nx + sx) + q];

    int sidex = (sx < 0) ? LEFT : RIGHT, sidey = (sy < 0) ? BOTTOM : TOP;
    int side;
    int qo = opp8(q);  /* the outgoing direction that is reflected into q */
    if (outx && outy) {
        int symx = o->el_type[sidex] == EL_SYMMETRY, symy = o->el_type[sidey] == EL_SYMMETRY;
        if (symx && symy) return gs[8 * (y * nx + x) + qo];   /* corner of two mirrors */
        side = symy ? sidex : sidey;
    } else {
        side = outx ? sidex : sidey;
        if (o->el_type[side] == EL_SYMMETRY) {
            /* mirror image across the wall (roller / symmetry plane) */
            if (outx) return gs[8 * (sy * nx + x) + find8(-C8X[q], C8Y[q])];
            return gs[8 * (y * nx + sx) + find8(C8X[q], -C8Y[q])];
        }
    }
    double d[2];
    if (o->el_type[side] == EL_DIRICHLET) {
        /* fullway bounce-back data term -6 w c.eta_D; the reflected population is
         * the post-collision one of the same pseudo-time step */
        link_data(o, nx, ny, lv->el_val[side], 2, side, x, y, C8X[qo], C8Y[qo], d);
        return gs[8 * (y * nx + x) + qo] - 6.0 * W8[qo] * (C8X[qo] * d[0] + C8Y[qo] * d[1]);
    }
    /* traction: halfway anti-bounce-back, eq. BC:traction */
    link_data(o, nx, ny, lv->el_val[side], 2, side, x, y, C8X[qo], C8Y[qo], d);
    return -gs[8 * (y * nx + x) + qo] + traction_term(side, q, d);
}

/* ELASTIC_STEP (Algorithm 2) on level lv: out = stream(collide(u, F)) with BCs */
static void elastic_step(const or_state *o, const level_t *lv, const double *u, const double *F,
                         double *gs_work, double *out)
{
#pragma omp parallel for schedule(static)
    for (int c = 0; c < lv->n; ++c) elastic_collide(o, u + 8 * c, F + 2 * c, gs_work + 8 * c);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < lv->ny; ++y)
        for (int x = 0; x < lv->nx; ++x)
            for (int q = 0; q < 8; ++q)
                out[8 * (y * lv->nx + x) + q] = elastic_incoming(o, lv, gs_work, x, y, q);
}

/* S(g) = ELASTIC_STEP(g - r, Ft + F_*(g)) as used in every line of Algorithm 4.
 * r may be NULL (zero), Ft may be NULL (zero). */
static void apply_S(const or_state *o, level_t *lv, const double *g, const double *r, const double *Ft,
                    double *out)
{
    int n = lv->n;
    self_force(o, lv, g, lv->D, lv->F);
    if (Ft) for (int c = 0; c < 2 * n; ++c) lv->F[c] += Ft[c];
    for (int c = 0; c < 8 * n; ++c) lv->u[c] = g[c] - (r ? r[c] : 0.0);
    elastic_step(o, lv, lv->u, lv->F, lv->gs, out);
}

/* S(g) of Algorithm 1 read with the lag of eq. source:implicit: the implicit
 * source, hence the self-force, takes the divergence of the previous
 * pseudo-time step's iterate (kept in Dlag), which then becomes the
 * divergence of g.  A time step starts with Dlag = D(g) (g(-1) = g(0)), where
 * this equals apply_S bitwise. */
static void apply_S_lagged(const or_state *o, level_t *lv, const double *g, const double *r, const double *Ft,
                           double *out)
{
    int n = lv->n;
    grad_central(o, lv->nx, lv->ny, o->Dlag, lv->F);
    for (int c = 0; c < 2 * n; ++c) lv->F[c] *= o->cstar;
    if (Ft) for (int c = 0; c < 2 * n; ++c) lv->F[c] += Ft[c];
    for (int c = 0; c < 8 * n; ++c) lv->u[c] = g[c] - (r ? r[c] : 0.0);
    elastic_step(o, lv, lv->u, lv->F, lv->gs, out);
    for (int c = 0; c < n; ++c) o->Dlag[c] = divergence_of(o, g + 8 * c);
}

/* start of a lagged pseudo-time run: g(-1) = g(0) */
static void lag_reset(const or_state *o, const level_t *lv, const double *g)
{
    for (int c = 0; c < lv->n; ++c) o->Dlag[c] = divergence_of(o, g + 8 * c);
}

/* one under-relaxed smoothing step, eq. MG:smoother */
static void smooth(const or_state *o, level_t *lv, double *g, const double *r, const double *Ft)
{
    if (o->Dlag)
        apply_S_lagged(o, lv, g, r, Ft, lv->S);
    else
        apply_S(o, lv, g, r, Ft, lv->S);
    for (int c = 0; c < 8 * lv->n; ++c) g[c] = (1.0 - o->gamma) * g[c] + o->gamma * lv->S[c];
}

/* ELASTIC_MULTIGRID (Algorithm 4) on level l; g is updated in place.
 *
 * cyc selects how often the coarse correction visits level l - 1.  The paper
 * gives the V-cycle (one visit) and names W- and F-cycles as future work
 * without defining them; these follow the textbook recursions:
 *   V: one V-visit;
 *   W: two W-visits, the second continuing from the first's coarse iterate
 *      with the same coarse right-hand side;
 *   F: an F-visit, then a V-visit continuing from its result.
 * On the coarsest level (no recursion) every shape is the same 2K sweeps. */
enum { CYC_V = 0, CYC_W = 1, CYC_F = 2, CYC_FMG = 3 };

/* residual g - g** of level l (eq. LBM:residual) summed over each 2x2 block
 * into the right-hand side of level l - 1 (eq. MG:restriction) */
static void restrict_residual(or_state *o, int l, const double *g, const double *r, const double *Ft)
{
    level_t *lv = &o->lv[l], *lc = &o->lv[l - 1];
    apply_S(o, lv, g, r, Ft, lv->S);
    memset(lc->r, 0, sizeof(double) * 8 * lc->n);
    for (int y = 0; y < lv->ny; ++y)
        for (int x = 0; x < lv->nx; ++x) {
            int cf = y * lv->nx + x, cc = (y / 2) * lc->nx + (x / 2);
            for (int q = 0; q < 8; ++q) lc->r[8 * cc + q] += g[8 * cf + q] - lv->S[8 * cf + q];
        }
}

/* prolongation P = R^T: every fine cell of level l adds its coarse cell's value */
static void prolong_add(or_state *o, int l, double *g)
{
    level_t *lv = &o->lv[l], *lc = &o->lv[l - 1];
    for (int y = 0; y < lv->ny; ++y)
        for (int x = 0; x < lv->nx; ++x) {
            int cf = y * lv->nx + x, cc = (y / 2) * lc->nx + (x / 2);
            for (int q = 0; q < 8; ++q) g[8 * cf + q] += lc->g[8 * cc + q];
        }
}

static void elastic_mg(or_state *o, int l, double *g, const double *r, const double *Ft, int cyc)
{
    level_t *lv = &o->lv[l];
    if (l == 1 && o->L > 1 && o->pb.coarse_sweeps > 0) {
        /* the coarsest level of a hierarchy with its own number of sweeps
         * (Algorithm 4 without recursion is 2K of them) */
        ++o->coarsest_visits;
        for (int k = 0; k < o->pb.coarse_sweeps; ++k) smooth(o, lv, g, r, Ft);
        return;
    }
    if (l == 1) ++o->coarsest_visits;
    for (int k = 0; k < o->K; ++k) smooth(o, lv, g, r, Ft);
    if (l > 1) {
        level_t *lc = &o->lv[l - 1];
        restrict_residual(o, l, g, r, Ft);
        /* coarse correction from zero with the coarse residual, no explicit force */
        memset(lc->g, 0, sizeof(double) * 8 * lc->n);
        elastic_mg(o, l - 1, lc->g, lc->r, NULL, cyc);
        if (cyc != CYC_V) elastic_mg(o, l - 1, lc->g, lc->r, NULL, cyc == CYC_W ? CYC_W : CYC_V);
        prolong_add(o, l, g);
    }
    for (int k = 0; k < o->K; ++k) smooth(o, lv, g, r, Ft);
}

/* Full multigrid (the conclusion names it as future work without defining
 * it), as the coarse-grid correction of a cycle.  fmg_solve computes the
 * correction of level l from zero by nested iteration: the residual of the
 * zero iterate (with the level's right-hand side) is restricted, the coarser
 * correction is computed the same way, prolongated as the starting iterate,
 * and one V-cycle on level l follows; on the coarsest level the correction
 * is its smoothing sweeps from zero.  fmg_cycle is Algorithm 4 with that
 * correction in place of the V-visit: K smoothing steps on the iterate (the
 * warm start of the time step), its restricted residual, the correction by
 * fmg_solve one level down, prolongation, K smoothing steps.  On one or two
 * levels it is the V-cycle. */
static void fmg_solve(or_state *o, int l, double *e, const double *r)
{
    if (l > 1) {
        level_t *lc = &o->lv[l - 1];
        restrict_residual(o, l, e, r, NULL);
        memset(lc->g, 0, sizeof(double) * 8 * lc->n);
        fmg_solve(o, l - 1, lc->g, lc->r);
        prolong_add(o, l, e);
    }
    elastic_mg(o, l, e, r, NULL, CYC_V);
}

static void fmg_cycle(or_state *o, int l, double *g, const double *r, const double *Ft)
{
    level_t *lv = &o->lv[l];
    if (l == 1) {
        elastic_mg(o, l, g, r, Ft, CYC_V);
        return;
    }
    level_t *lc = &o->lv[l - 1];
    for (int k = 0; k < o->K; ++k) smooth(o, lv, g, r, Ft);
    restrict_residual(o, l, g, r, Ft);
    memset(lc->g, 0, sizeof(double) * 8 * lc->n);
    fmg_solve(o, l - 1, lc->g, lc->r);
    prolong_add(o, l, g);
    for (int k = 0; k < o->K; ++k) smooth(o, lv, g, r, Ft);
}

/* cycle j (from 0) of a time step: full multigrid takes the first */
static void step_cycle(or_state *o, int j)
{
    if (o->pb.cycle == CYC_FMG && j == 0)
        fmg_cycle(o, o->L, o->g, NULL, o->Ft);
    else
        elastic_mg(o, o->L, o->g, NULL, o->Ft, o->pb.cycle == CYC_FMG ? CYC_V : o->pb.cycle);
}

/* ---------------------------------------------------------------- flow */
static double flow_incoming(const or_state *o, const double *fs, int x, int y, int i)
{
    int nx = o->nx, ny = o->ny;
    if (i == 0) return fs[9 * (y * nx + x)];
    int sx = x - C9X[i], sy = y - C9Y[i];
    int outx = (sx < 0 || sx >= nx), outy = (sy < 0 || sy >= ny);
    if (outx && side_periodic(o, LEFT)) { sx = wrapi(sx, nx); outx = 0; }
    if (outy && side_periodic(o, BOTTOM)) { sy = wrapi(sy, ny); outy = 0; }
    if (!outx && !outy) return fs[9 * (sy * nx + sx) + i];
    int sidex = (sx < 0) ? LEFT : RIGHT, sidey = (sy < 0) ? BOTTOM : TOP;
    int tx = o->flow_type[sidex] ? o->flow_type[sidex][y] : 0;
    int ty = o->flow_type[sidey] ? o->flow_type[sidey][x] : 0;
    int side, type;
    int io = opp9(i);
    if (outx && outy) {
        int symx = (tx == FL_SYMMETRY), symy = (ty == FL_SYMMETRY);
        if (symx && symy) return fs[9 * (y * nx + x) + io];
        if (symy) { side = sidex; type = tx; } else { side = sidey; type = ty; }
    } else if (outx) {
        side = sidex; type = tx;
        if (type == FL_SYMMETRY) return fs[9 * (sy * nx + x) + find9(-C9X[i], C9Y[i])];
    } else {
        side = sidey; type = ty;
        if (type == FL_SYMMETRY) return fs[9 * (y * nx + sx) + find9(C9X[i], -C9Y[i])];
    }
    if (type == FL_NOFLOW) return fs[9 * (y * nx + x) + io];       /* eq. BC:noFlow */
    /* Dirichlet: halfway anti-bounce-back, eq. BC:pressure */
    double pd;
    link_data(o, nx, ny, o->p_bc[side], 1, side, x, y, C9X[io], C9Y[io], &pd);
    return -fs[9 * (y * nx + x) + io] + 2.0 * W9[io] * pd;
}

/* FLOW_STEP (Algorithm 3) with the effective source s (lattice units) */
static void flow_step(or_state *o, const double *s, double *fs_work)
{
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->n; ++c) {
        const double *fc = o->f + 9 * c;
        double om = o->om_f[c];
        double p = 0.0;
        for (int i = 0; i < 9; ++i) p += fc[i];
        p += 0.5 * s[c];                                        /* eq. pressure */
        for (int i = 0; i < 9; ++i) {
            double feq = W9[i] * p;                             /* eq. pressure:equilibrium */
            double Si = (1.0 - 0.5 * om) * W9[i] * s[c];        /* eq. pressure:collision:source */
            fs_work[9 * c + i] = fc[i] - om * (fc[i] - feq) + Si;   /* eq. pressure:collision */
        }
    }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < o->ny; ++y)
        for (int x = 0; x < o->nx; ++x)
            for (int i = 0; i < 9; ++i) o->f[9 * (y * o->nx + x) + i] = flow_incoming(o, fs_work, x, y, i);
}

/* ------------------------------------------------------- coupling pieces */
/* explicit part of the centred source, eq. source:implicit without the term of
 * the current pseudo-time iterate */
static void explicit_source(const or_state *o, double *st)
{
    for (int c = 0; c < o->n; ++c)
        st[c] = o->src[c] - (o->alpha / o->h) * ((1.0 - o->r) * (o->D1[c] - o->D2[c]) - o->r * o->D1[c]);
}

/* explicit force Ft = h^2 c0 f - alpha h grad p, with the explicit source part.
 * The gradient is either the first-moment form of eq. pressure:gradient,
 *   grad p = -3 omega sum_i f_i c_i + (1/2) grad^c s,
 * or the central difference of eq. pressure:gradient:alternative applied to
 * p = sum_i f_i + s/2 (eq. pressure), i.e. grad^c(sum_i f_i) + (1/2) grad^c s;
 * the s part, which carries the implicit coupling, is the same in both. */
static void explicit_force(or_state *o, double *st, double *gst)
{
    explicit_source(o, st);
    grad_central(o, o->nx, o->ny, st, gst);
    double *gP = NULL;
    if (o->pb.pressure_gradient == 1) {
        double *P0 = (double *)malloc(sizeof(double) * o->n);
        gP = (double *)malloc(sizeof(double) * 2 * o->n);
        for (int c = 0; c < o->n; ++c) {
            double s = 0.0;
            for (int i = 0; i < 9; ++i) s += o->f[9 * c + i];
            P0[c] = s;
        }
        grad_central(o, o->nx, o->ny, P0, gP);
        free(P0);
    }
    for (int c = 0; c < o->n; ++c) {
        double gpx, gpy;
        if (gP) {
            gpx = gP[2 * c] + 0.5 * gst[2 * c];
            gpy = gP[2 * c + 1] + 0.5 * gst[2 * c + 1];
        } else {
            const double *fc = o->f + 9 * c;
            double jx = 0.0, jy = 0.0;
            for (int i = 0; i < 9; ++i) { jx += fc[i] * C9X[i]; jy += fc[i] * C9Y[i]; }
            double om = o->om_f[c];
            gpx = -3.0 * om * jx + 0.5 * gst[2 * c];
            gpy = -3.0 * om * jy + 0.5 * gst[2 * c + 1];
        }
        o->Ft[2 * c] = o->fbody[2 * c] - o->alpha * o->h * gpx;
        o->Ft[2 * c + 1] = o->fbody[2 * c + 1] - o->alpha * o->h * gpy;
    }
    free(gP);
}

static double sumsq(const double *a, long n)
{
    double s = 0.0;
    for (long k = 0; k < n; ++k) s += a[k] * a[k];
    return s;
}

/* --------------------------------------------------------------- lifecycle */
static void free_state(or_state *o)
{
    if (!o) return;
    if (o->lv) {
        for (int l = 1; l <= o->L; ++l) {
            level_t *lv = &o->lv[l];
            for (int s = 0; s < 4; ++s) free(lv->el_val[s]);
            free(lv->g); free(lv->r); free(lv->u); free(lv->F); free(lv->D); free(lv->gs);
            free(lv->S); free(lv->tmp);
        }
        free(o->lv);
    }
    for (int s = 0; s < 4; ++s) { free(o->flow_type[s]); free(o->p_bc[s]); }
    free(o->om_f); free(o->f); free(o->g); free(o->D1); free(o->D2); free(o->Ft);
    free(o->fbody); free(o->src); free(o->eta); free(o->p); free(o->sig);
    free(o->ne_hist); free(o->ratio_hist); free(o->Dlag);
    free(o);
}

int or_default_levels(int nx, int ny)
{
    int L = 1;
    while (nx % 2 == 0 && ny % 2 == 0 && nx / 2 >= 2 && ny / 2 >= 2) { nx /= 2; ny /= 2; ++L; }
    return L;
}

static void set_initial(or_state *o);

or_state *or_create(const or_problem *pb, int *err)
{
    *err = OR_ERR_ARG;
    if (pb->nx < 1 || pb->ny < 1 || pb->dx <= 0 || pb->dt <= 0 || pb->c0 <= 0 || pb->mu <= 0 ||
        pb->lambda + pb->mu <= 0 || pb->alpha < 0 || pb->alpha > 1 || pb->r < 0 || pb->r > 1 ||
        pb->gamma <= 0 || pb->gamma > 1 || pb->K < 1 || pb->pressure_gradient < 0 || pb->pressure_gradient > 1 ||
        pb->cycle < 0 || pb->cycle > 3 || pb->fstar_literal < 0 || pb->fstar_literal > 1 ||
        pb->coarse_sweeps < 0 || pb->coarse_sweeps % 2 != 0 || pb->lag < 0 || pb->lag > 1)
        return NULL;
    for (int s = 0; s < 4; ++s) if (pb->el_type[s] < 0 || pb->el_type[s] > 3) return NULL;
    if ((pb->el_type[LEFT] == EL_PERIODIC) != (pb->el_type[RIGHT] == EL_PERIODIC)) return NULL;
    if ((pb->el_type[BOTTOM] == EL_PERIODIC) != (pb->el_type[TOP] == EL_PERIODIC)) return NULL;
    int L = pb->levels > 0 ? pb->levels : or_default_levels(pb->nx, pb->ny);
    if (pb->nx % (1 << (L - 1)) || pb->ny % (1 << (L - 1))) return NULL;
    if (L > 1 && (pb->nx >> (L - 1) < 1 || pb->ny >> (L - 1) < 1)) return NULL;
    if (pb->lag && (L != 1 || pb->ne_fixed < 1)) return NULL;   /* Algorithm 1 with fixed N_E only */

    or_state *o = (or_state *)calloc(1, sizeof(or_state));
    if (!o) { *err = OR_ERR_NOMEM; return NULL; }
    o->pb = *pb;
    o->nx = pb->nx; o->ny = pb->ny; o->n = pb->nx * pb->ny; o->L = L; o->K = pb->K;
    o->h = pb->dx; o->dt = pb->dt; o->gamma = pb->gamma; o->r = pb->r; o->alpha = pb->alpha;
    o->c0 = pb->c0;
    o->lam = pb->c0 * pb->lambda;
    o->mu = pb->c0 * pb->mu;
    /* Table 2 rates and the derived factors of eqs. moments:bared, moments:collision:22 */
    o->om_s = 2.0 / (3.0 * (o->lam + o->mu) + 1.0);
    o->om_d = 2.0 / (6.0 * o->mu + 1.0);
    o->b_s = 3.0 * (o->lam + o->mu) / (3.0 * (o->lam + o->mu) + 1.0);
    o->b_d = 6.0 * o->mu / (6.0 * o->mu + 1.0);
    o->beta22 = 1.0 / (12.0 * (o->lam + o->mu) + 4.0);
    o->cstar = (pb->fstar_literal ? 1.0 : o->r) * o->alpha * o->alpha / 2.0;
    int n = o->n;
    o->om_f = (double *)malloc(sizeof(double) * n);
    for (int c = 0; c < n; ++c) {
        double kap = pb->kappa ? pb->kappa[c] : pb->kappa_uniform;
        if (!(kap > 0)) { free_state(o); return NULL; }
        double k = (kap / pb->c0) * pb->dt / (pb->dx * pb->dx);   /* lattice diffusivity */
        o->om_f[c] = 1.0 / (3.0 * k + 0.5);                        /* eq. pressure:rate */
    }
    for (int s = 0; s < 4; ++s) {
        int len = (s == LEFT || s == RIGHT) ? o->ny : o->nx;
        o->el_type[s] = pb->el_type[s];
        o->flow_type[s] = (int8_t *)malloc(len);
        o->p_bc[s] = (double *)calloc(len, sizeof(double));
        for (int k = 0; k < len; ++k) {
            o->flow_type[s][k] = pb->flow_type[s] ? pb->flow_type[s][k] : 0;
            if (pb->p_value[s]) o->p_bc[s][k] = pb->c0 * pb->p_value[s][k];
            int periodic_side = (o->el_type[s] == EL_PERIODIC);
            if (periodic_side != (o->flow_type[s][k] == FL_PERIODIC)) { free_state(o); return NULL; }
        }
    }
    o->lv = (level_t *)calloc(L + 1, sizeof(level_t));
    for (int l = L; l >= 1; --l) {
        level_t *lv = &o->lv[l];
        lv->nx = o->nx >> (L - l); lv->ny = o->ny >> (L - l); lv->n = lv->nx * lv->ny;
        int m = lv->n;
        lv->g = calloc(8 * m, sizeof(double)); lv->r = calloc(8 * m, sizeof(double));
        lv->u = calloc(8 * m, sizeof(double)); lv->F = calloc(2 * m, sizeof(double));
        lv->D = calloc(m, sizeof(double)); lv->gs = calloc(8 * m, sizeof(double));
        lv->S = calloc(8 * m, sizeof(double)); lv->tmp = calloc(8 * m, sizeof(double));
        for (int s = 0; s < 4; ++s) {
            int len = (s == LEFT || s == RIGHT) ? lv->ny : lv->nx;
            lv->el_val[s] = calloc(2 * len, sizeof(double));
            if (l == L && pb->el_value[s]) {
                for (int k = 0; k < 2 * len; ++k) {
                    double v = pb->el_value[s][k];
                    /* traction enters as h * (c0 t); Dirichlet data are displacements */
                    lv->el_val[s][k] = (o->el_type[s] == EL_TRACTION) ? o->h * pb->c0 * v : v;
                }
            }
        }
    }
    o->f = calloc(9 * n, sizeof(double)); o->g = calloc(8 * n, sizeof(double));
    o->D1 = calloc(n, sizeof(double)); o->D2 = calloc(n, sizeof(double));
    o->Ft = calloc(2 * n, sizeof(double)); o->fbody = calloc(2 * n, sizeof(double));
    o->src = calloc(n, sizeof(double));
    o->eta = calloc(2 * n, sizeof(double)); o->p = calloc(n, sizeof(double));
    o->sig = calloc(3 * n, sizeof(double));
    o->hist_cap = 0;
    o->threads = 1;
    if (pb->lag) o->Dlag = calloc(n, sizeof(double));
    set_initial(o);
    *err = OR_OK;
    return o;
}

void or_destroy(or_state *o) { free_state(o); }

/* loads at the time of the next step, dimensional: body force f (2 x N, component
 * planes) and fluid source s (N); NULL means zero */
int or_set_loads(or_state *o, const double *body_f, const double *source_s, int reinit)
{
    int n = o->n;
    for (int c = 0; c < n; ++c) {
        o->fbody[2 * c] = body_f ? o->h * o->h * o->c0 * body_f[c] : 0.0;
        o->fbody[2 * c + 1] = body_f ? o->h * o->h * o->c0 * body_f[n + c] : 0.0;
        o->src[c] = source_s ? o->dt * source_s[c] : 0.0;
    }
    if (reinit) set_initial(o);
    return OR_OK;
}

/* initial conditions, eqs. ICs and ICs:moments with p = 0 and eta = 0 at t = 0
 * (so the effective force is the body force alone) */
static void set_initial(or_state *o)
{
    for (int c = 0; c < o->n; ++c) {
        for (int i = 0; i < 9; ++i) o->f[9 * c + i] = -0.5 * W9[i] * o->src[c];
        double F0[2] = {o->fbody[2 * c], o->fbody[2 * c + 1]};
        double m0[8] = {0};
        m0[T_M10] = -0.5 * F0[0]; m0[T_M01] = -0.5 * F0[1];
        m0[T_M12] = -F0[0] / 6.0; m0[T_M21] = -F0[1] / 6.0;
        for (int q = 0; q < 8; ++q) {
            double v = 0.0;
            for (int k = 0; k < 8; ++k) v += TAB3[q][k] * m0[k];
            o->g[8 * c + q] = v;
        }
        o->D1[c] = 0.0; o->D2[c] = 0.0;
    }
    o->step = 0;
    o->status = OR_OK;
}

/* outputs from the current populations and force, eqs. displacement,
 * moments:bared; stress is returned in physical units sigma = sigma_lat/(c0 h) */
static void extract(or_state *o, const double *s_now)
{
    level_t *lv = &o->lv[o->L];
    self_force(o, lv, o->g, lv->D, lv->F);
    int n = o->n;
    for (int c = 0; c < n; ++c) {
        const double *gc = o->g + 8 * c;
        double Fx = o->Ft[2 * c] + lv->F[2 * c], Fy = o->Ft[2 * c + 1] + lv->F[2 * c + 1];
        o->eta[c] = raw_moment(gc, 1, 0) + 0.5 * Fx;
        o->eta[n + c] = raw_moment(gc, 0, 1) + 0.5 * Fy;
        double m20 = raw_moment(gc, 2, 0), m02 = raw_moment(gc, 0, 2);
        double bms = o->b_s * (m20 + m02), bmd = o->b_d * (m20 - m02), bm11 = o->b_d * raw_moment(gc, 1, 1);
        double sc = 1.0 / (o->c0 * o->h);
        o->sig[c] = -0.5 * (bms + bmd) * sc;
        o->sig[n + c] = -bm11 * sc;
        o->sig[2 * n + c] = -0.5 * (bms - bmd) * sc;
        double p = 0.0;
        for (int i = 0; i < 9; ++i) p += o->f[9 * c + i];
        o->p[c] = (p + 0.5 * s_now[c]) / o->c0;                 /* eq. pressure */
    }
}

static int finite_all(const double *a, long n)
{
    for (long k = 0; k < n; ++k) if (!isfinite(a[k])) return 0;
    return 1;
}

/* one coupled time step, Algorithm 5 */
static int one_step(or_state *o)
{
    int n = o->n;
    level_t *lv = &o->lv[o->L];
    double *st = (double *)malloc(sizeof(double) * n);
    double *gst = (double *)malloc(sizeof(double) * 2 * n);
    double *fs = (double *)malloc(sizeof(double) * 9 * n);
    double *Dn = (double *)malloc(sizeof(double) * n);
    double *sn = (double *)malloc(sizeof(double) * n);

    /* explicit part of the source and the explicit force */
    explicit_force(o, st, gst);

    /* elasticity: N_E multigrid cycles (fixed, replayed or adaptive) */
    int ne_fixed = o->pb.ne_fixed;
    if (o->ne_sched && o->step < o->ne_sched_len) ne_fixed = o->ne_sched[o->step];
    int j = 0;
    double ratio = -1.0;
    if (o->Dlag) lag_reset(o, lv, o->g);
    if (ne_fixed > 0) {
        for (j = 0; j < ne_fixed; ++j) step_cycle(o, j);
    } else {
        /* adaptive: before each cycle the residual of the current iterate is
         * compared with the iterate itself (stop when ||g - S(g)|| <= tol ||g||,
         * at least one cycle, at most ne_max) */
        for (;;) {
            apply_S(o, lv, o->g, NULL, o->Ft, lv->tmp);
            for (int c = 0; c < 8 * n; ++c) lv->tmp[c] = o->g[c] - lv->tmp[c];
            double nr = sqrt(sumsq(lv->tmp, 8L * n)), ng = sqrt(sumsq(o->g, 8L * n));
            ratio = ng > 0 ? nr / ng : 0.0;
            if (!isfinite(nr)) break;
            if (j >= 1 && nr <= o->pb.ne_tol * ng) break;
            if (j >= o->pb.ne_max) break;
            step_cycle(o, j);
            ++j;
        }
    }
    if (o->hist_cap > o->step) { o->ne_hist[o->step] = j; o->ratio_hist[o->step] = ratio; }

    /* divergence after the solve, then the centred source of the flow update */
    for (int c = 0; c < n; ++c) Dn[c] = divergence_of(o, o->g + 8 * c);
    for (int c = 0; c < n; ++c)
        sn[c] = o->src[c] - (o->alpha / o->h) * ((1.0 - o->r) * (o->D1[c] - o->D2[c]) + o->r * (Dn[c] - o->D1[c]));
    extract(o, sn);
    flow_step(o, sn, fs);
    memcpy(o->D2, o->D1, sizeof(double) * n);
    memcpy(o->D1, Dn, sizeof(double) * n);
    o->step += 1;
    int ok = finite_all(o->g, 8L * n) && finite_all(o->f, 9L * n);
    free(st); free(gst); free(fs); free(Dn); free(sn);
    return ok ? OR_OK : OR_ERR_DIVERGED;
}

int or_step(or_state *o, int nsteps)
{
    if (o->status != OR_OK) return OR_ERR_STATE;
#ifdef _OPENMP
    omp_set_num_threads(o->threads > 0 ? o->threads : 1);
#endif
    for (int k = 0; k < nsteps; ++k) {
        int rc = one_step(o);
        if (rc != OR_OK) { o->status = rc; return rc; }
    }
    return OR_OK;
}

int or_set_threads(or_state *o, int threads) { o->threads = threads; return OR_OK; }

int or_set_history(or_state *o, int cap)
{
    free(o->ne_hist); free(o->ratio_hist);
    o->ne_hist = calloc(cap > 0 ? cap : 1, sizeof(int));
    o->ratio_hist = calloc(cap > 0 ? cap : 1, sizeof(double));
    o->hist_cap = cap;
    return OR_OK;
}

int or_get_history(const or_state *o, int *ne, double *ratio, int cap)
{
    int m = cap < o->hist_cap ? cap : o->hist_cap;
    if (m > o->step) m = o->step;
    for (int k = 0; k < m; ++k) { ne[k] = o->ne_hist[k]; ratio[k] = o->ratio_hist[k]; }
    return m;
}

/* replay a given number of cycles per step (index = step number) */
int or_set_ne_schedule(or_state *o, const int *ne, int len) { o->ne_sched = ne; o->ne_sched_len = len; return OR_OK; }

/* fields of the last completed step: eta (2 x N), p (N), sigma (3 x N: 11, 12, 22) */
int or_get_fields(const or_state *o, double *eta, double *p, double *sigma, int *step)
{
    int n = o->n;
    if (eta) memcpy(eta, o->eta, sizeof(double) * 2 * n);
    if (p) memcpy(p, o->p, sizeof(double) * n);
    if (sigma) memcpy(sigma, o->sig, sizeof(double) * 3 * n);
    if (step) *step = o->step;
    return o->status;
}

/* ---- state access for single-operation checks; populations are given as
 * component planes: f (9 x N), g (8 x N) */
int or_get_state(const or_state *o, double *f, double *g, double *D1, double *D2, int *step)
{
    int n = o->n;
    for (int c = 0; c < n; ++c) {
        if (f) for (int i = 0; i < 9; ++i) f[i * n + c] = o->f[9 * c + i];
        if (g) for (int q = 0; q < 8; ++q) g[q * n + c] = o->g[8 * c + q];
    }
    if (D1) memcpy(D1, o->D1, sizeof(double) * n);
    if (D2) memcpy(D2, o->D2, sizeof(double) * n);
    if (step) *step = o->step;
    return OR_OK;
}

int or_set_state(or_state *o, const double *f, const double *g, const double *D1, const double *D2, int step)
{
    int n = o->n;
    for (int c = 0; c < n; ++c) {
        if (f) for (int i = 0; i < 9; ++i) o->f[9 * c + i] = f[i * n + c];
        if (g) for (int q = 0; q < 8; ++q) o->g[8 * c + q] = g[q * n + c];
    }
    if (D1) memcpy(o->D1, D1, sizeof(double) * n);
    if (D2) memcpy(o->D2, D2, sizeof(double) * n);
    o->step = step;
    o->status = OR_OK;
    return OR_OK;
}

/* explicit force of the current state (2 x N planes, lattice units) */
int or_explicit_force(or_state *o, double *Ft_planes)
{
    int n = o->n;
    double *st = malloc(sizeof(double) * n), *gst = malloc(sizeof(double) * 2 * n);
    explicit_force(o, st, gst);
    for (int c = 0; c < n; ++c) { Ft_planes[c] = o->Ft[2 * c]; Ft_planes[n + c] = o->Ft[2 * c + 1]; }
    free(st); free(gst);
    return OR_OK;
}

static void planes_to_aos(const double *pl, double *aos, int n, int m)
{ for (int c = 0; c < n; ++c) for (int k = 0; k < m; ++k) aos[m * c + k] = pl ? pl[k * n + c] : 0.0; }
static void aos_to_planes(const double *aos, double *pl, int n, int m)
{ for (int c = 0; c < n; ++c) for (int k = 0; k < m; ++k) pl[k * n + c] = aos[m * c + k]; }

/* one application S(g) = ELASTIC_STEP(g - r, Ft + F_*(g)) on level l (l = L is the
 * finest, with the problem's boundary data; coarser levels use homogeneous data).
 * Arrays are component planes of that level's size; r and Ft may be NULL. */
int or_apply_elastic(or_state *o, int l, const double *g, const double *r, const double *Ft, double *out)
{
    if (l < 1 || l > o->L) return OR_ERR_ARG;
    level_t *lv = &o->lv[l];
    int m = lv->n;
    double *ga = malloc(sizeof(double) * 8 * m), *ra = malloc(sizeof(double) * 8 * m);
    double *fa = malloc(sizeof(double) * 2 * m), *oa = malloc(sizeof(double) * 8 * m);
    planes_to_aos(g, ga, m, 8); planes_to_aos(r, ra, m, 8); planes_to_aos(Ft, fa, m, 2);
    apply_S(o, lv, ga, r ? ra : NULL, Ft ? fa : NULL, oa);
    aos_to_planes(oa, out, m, 8);
    free(ga); free(ra); free(fa); free(oa);
    return OR_OK;
}

/* one ELASTIC_MULTIGRID cycle on level l with rhs r and force Ft (planes) */
int or_mg_cycle(or_state *o, int l, double *g, const double *r, const double *Ft)
{
    if (l < 1 || l > o->L) return OR_ERR_ARG;
    level_t *lv = &o->lv[l];
    int m = lv->n;
    double *ga = malloc(sizeof(double) * 8 * m), *ra = malloc(sizeof(double) * 8 * m);
    double *fa = malloc(sizeof(double) * 2 * m);
    planes_to_aos(g, ga, m, 8); planes_to_aos(r, ra, m, 8); planes_to_aos(Ft, fa, m, 2);
    /* the recursion uses the level's own g buffer; work on a private copy.
     * Full multigrid runs its first cycle; the lagged Algorithm 1 starts as a
     * time step does (g(-1) = g(0)). */
    if (o->Dlag) lag_reset(o, lv, ga);
    if (o->pb.cycle == CYC_FMG)
        fmg_cycle(o, l, ga, r ? ra : NULL, Ft ? fa : NULL);
    else
        elastic_mg(o, l, ga, r ? ra : NULL, Ft ? fa : NULL, o->pb.cycle);
    aos_to_planes(ga, g, m, 8);
    free(ga); free(ra); free(fa);
    return OR_OK;
}

/* coarsest-level solves since creation */
long or_coarsest_visits(const or_state *o) { return o->coarsest_visits; }

/* level sizes */
int or_level_shape(const or_state *o, int l, int *nx, int *ny)
{
    if (l < 1 || l > o->L) return OR_ERR_ARG;
    *nx = o->lv[l].nx; *ny = o->lv[l].ny;
    return o->L;
}

/* one FLOW_STEP on the current f with the given lattice source (N values) */
int or_flow_step(or_state *o, const double *s_lat)
{
    double *fs = malloc(sizeof(double) * 9 * o->n);
    flow_step(o, s_lat, fs);
    free(fs);
    return OR_OK;
}
