/*
 * FP64 CPU oracle of the coupled lattice Boltzmann model of aqueous-humour dynamics
 * (Qin, Meng, Yang, Zhang & Wen, "Aqueous humor dynamics in human eyes: a lattice
 * Boltzmann study", arXiv:2102.12663).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct statement of
 * what one time step computes.  It is used by the tests, by the smoke check and by the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code, header or
 * constant table with the HIP library.
 *
 * Form: push.  Each step (1) collides every active node, then (2) streams every
 * post-collision population to its downstream neighbour or, at a link into a non-active
 * node, applies that link's boundary rule, then (3) swaps the buffers.  Every step is
 * taken in the paper's order and notation:
 *
 *   flow     f_i(x+e_i, t+1) = f_i - (f_i - f_i^eq)/tau + F_i            (eq. 6)
 *            f_i^eq = lambda_i p + S_i(u), lambda_{1-4}=lambda, lambda_{5-8}=gamma (eq. 7)
 *            S_i(u) = w_i [3 e_i.u + 9/2 (e_i.u)^2 - 3/2 |u|^2]            (eq. 8)
 *            u = sum_i e_i f_i,  p = c^2/(4 sigma) [sum_{i>=1} f_i + S_0(u)] (eq. 9)
 *   thermal  T_i(x+e_i, t+1) = T_i - (T_i - T_i^eq)/tau_T                 (eq. 11)
 *            T_i^eq = w^T_i T [1 + e_i.u / c_sT^2]                        (eq. 12, D2Q5)
 *            T = sum_i T_i                                                 (eq. 13)
 *   force    F = g beta (T - T0) (sin phi, cos phi), i.e. -g beta (T-T0) with gravity
 *            g = |g| (-sin phi, -cos phi)                                 (eq. 15-16)
 *            F_i = 1/2 e_i.F on the four axis links, 0 on diagonals       (eq. 17)
 *   Darcy    in POROUS nodes the drag F_D = -(nu/K) u_D, with the mid-step
 *            velocity u_D = (u + F_b/2) / (1 + nu/(2K)), enters as
 *            3 w_i e_i.F_D on every link                                  (eq. 4)
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - sigma = 5/12, lambda = 1/3, gamma = 1/12: the unique choice with lambda_i = 3 w_i,
 *     satisfying the constraints printed under eq. 7.
 *   - The state is held as deviations h_i = f_i - lambda_i p_ref (i = 1..8) and
 *     g_i = T_i - w^T_i T_ref (i = 0..4).  This is an exact affine change of variables
 *     (sum_{i>=1} lambda_i = 4 sigma, sum_i e_i lambda_i = 0), so eq. 6-13 keep their form:
 *     u = sum e_i h_i, p - p_ref = c^2/(4 sigma)[sum h_i + S_0(u)],
 *     h_i^eq = lambda_i (p - p_ref) + S_i(u).  It keeps the small pressure signal from
 *     cancelling against p_ref = 1/3.
 *   - f_0 is not carried: it enters neither u nor p (eq. 9 sums i >= 1 and e_0 = 0).
 *   - Thermal lattice D2Q5 with rest weight w0 and w^T_{1-4} = (1-w0)/4, c_sT^2 =
 *     (1-w0)/2; w0 = 0 is the paper's D2Q4 exactly (eq. 11-14).
 *   - Gravity at an angle: alpha_i = 1 on all four axis links (reduces to eq. 17 when
 *     gravity is along y).
 *   - Boundaries are link-wise: half-way bounce-back at SOLID, moving-wall bounce-back
 *     at INLET (wall velocity u_in), anti-bounce-back pressure at OUTLET (p_out, the
 *     O(u^2) term dropped).  Thermal: anti-bounce-back Dirichlet at CORNEA, IRIS and
 *     INLET (T_cornea, T_iris, T_inlet), adiabatic bounce-back at BOX and OUTLET.
 *   - The paper's wall scheme (bc_scheme = 1, section 2.3: Bouzidi et al.): a population
 *     leaving fluid node x along e_o toward a CORNEA or IRIS wall that the link meets at the
 *     fraction q of its length returns along e_i = -e_o as the linear interpolation
 *     q < 1/2:  2q f*_o(x) + (1 - 2q) f*_o(x - e_o)
 *     q >= 1/2: f*_o(x) / (2q) + (2q - 1)/(2q) f*_i(x)
 *     (f* post-collision); q = 1/2 is the half-way bounce-back.  Where q < 1/2 and x - e_o
 *     is not an active node the half-way bounce-back is kept.
 *     Inlet and outlet (section 2.3: Guo et al.'s non-equilibrium extrapolation): the
 *     population entering fluid node x from an INLET or OUTLET node b along e_i is b's
 *     post-collision value, the equilibrium of b's state plus the non-equilibrium part of
 *     x's post-collision population along e_i:
 *         f_i = f^eq_i(p_b, u_b) + [f*_i(x) - f^eq_i(p*, u*)],
 *     (p*, u*) the moments of x's post-collision populations; INLET: u_b = u_in, p_b = p*;
 *     pressure OUTLET: p_b = p_out, u_b = u*; lumped OUTLET: u_b = u_s n, p_b = p*.
 *     Thermal Dirichlet walls and the inlet (section 2.3, the extrapolation method) likewise:
 *         T_i = T^eq_i(T_w, u_b) + [T*_i(x) - T^eq_i(T*, u*)],  u_b = u_in at INLET, 0 at
 *     walls, T* = sum of x's post-collision thermal populations.  The boundary node b is
 *     taken to lie on the boundary (one link from x).  At t = 0 these populations are those
 *     the rules give from the initial equilibrium.
 *   - Lumped meshwork outlet (the coupling of section 2.2.4 with eq. 2 and eq. 4): the
 *     pressure in the meshwork falls linearly over its thickness h_TM from the IOP to the
 *     Schlemm's-canal pressure p_sc, so Darcy's law gives the seepage speed
 *     u_s = (K_TM / mu) (IOP - p_sc) / h_TM, with mu = nu (unit density) and IOP the mean
 *     pressure over FLUID nodes.  u_s is re-evaluated at every check step and holds for
 *     the next check interval; the first interval uses the initial pressure p_init.  OUTLET
 *     nodes then act as a wall moving at u_s along their outward direction n (stored in
 *     the wall bits: 0 +x, 1 +y, 2 -x, 3 -y): moving-wall bounce-back with that velocity.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so rounding follows
 * the written order).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "aq_oracle.h"

/* Threads of the OpenMP loops (timing of the oracle at a chosen thread count). */
void or_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}
int or_max_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------- lattice (section 2.3) */
/* D2Q9 velocities: e_0 rest, e_1..e_4 axis, e_5..e_8 diagonal; e_2 and e_4 are the
 * y (gravity) axis of eq. 17. */
static const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int opposite[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* eq. 8 weights */
static double w_flow(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

/* eq. 7 constants: lambda + gamma = sigma, lambda + 2 gamma = 1/2 */
static const double sigma_ = 5.0 / 12.0;
static double lambda_i(int i) { return i <= 4 ? 1.0 / 3.0 : 1.0 / 12.0; }

static double w_heat(const or_params* P, int i) { return i == 0 ? P->w0 : (1.0 - P->w0) / 4.0; }

/* eq. 8: S_i(u), c = 1 */
static double S(int i, double ux, double uy)
{
    double eu = ex[i] * ux + ey[i] * uy;
    double uu = ux * ux + uy * uy;
    return w_flow(i) * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

/* ---------------------------------------------------------------- state */
struct or_state {
    or_params P;
    int nx, ny;
    size_t n;
    uint8_t* cls;
    uint8_t* wall;
    double* h;      /* [8][n] flow deviations, pre-collision, slot q-1 holds direction q */
    double* g;      /* [5][n] thermal deviations, pre-collision */
    double* hs;     /* post-collision / next buffers */
    double* gs;
    double* hn;
    double* gn;
    double* u_prev_x;
    double* u_prev_y;
    double* T_prev;
    int n_walls;
    int32_t* wall_node;
    double* wall_q;          /* [n_walls][8] link fractions */
    int32_t* wall_of;        /* [n] index into the wall list, -1 off it */
    int32_t* wall_id;
    double* wall_nx;
    double* wall_ny;
    double q_out_last, q_in_last;
    double u_seep;           /* lumped meshwork seepage speed in effect */
    double gx_hat, gy_hat;   /* (sin phi, cos phi): direction of the buoyant force for T > T0 */
    int64_t step;
    or_observables obs;
};

#define H(s, q, k) (s)->h[(size_t)((q) - 1) * (s)->n + (k)]
#define G(s, q, k) (s)->g[(size_t)(q) * (s)->n + (k)]

static int is_active(const or_state* s, size_t k) { return s->cls[k] == OR_FLUID || s->cls[k] == OR_POROUS; }

/* Neighbour of node (x, y) along (dx, dy); -1 if it leaves a non-periodic lattice. */
static long neighbour(const or_state* s, int x, int y, int dx, int dy)
{
    int xx = x + dx, yy = y + dy;
    if (s->P.periodic_x) xx = (xx + s->nx) % s->nx;
    if (s->P.periodic_y) yy = (yy + s->ny) % s->ny;
    if (xx < 0 || xx >= s->nx || yy < 0 || yy >= s->ny) return -1;
    return (long)yy * s->nx + xx;
}

/* ---------------------------------------------------------------- moments (eq. 9, 13) */
typedef struct { double dp, ux, uy, T; } moments;

static moments moments_of(const or_state* s, const double* h8, const double* g5)
{
    moments m;
    double sum = 0.0, ux = 0.0, uy = 0.0, T = 0.0;
    for (int i = 1; i <= 8; i++) {
        sum += h8[i - 1];
        ux += ex[i] * h8[i - 1];
        uy += ey[i] * h8[i - 1];
    }
    m.ux = ux;
    m.uy = uy;
    /* p - p_ref = c^2/(4 sigma) [sum_{i>=1} h_i + S_0(u)] */
    m.dp = (1.0 / (4.0 * sigma_)) * (sum + S(0, ux, uy));
    for (int i = 0; i <= 4; i++) T += g5[i];
    m.T = s->P.T_ref + T;
    return m;
}

static void gather(const or_state* s, size_t k, double* h8, double* g5)
{
    for (int i = 1; i <= 8; i++) h8[i - 1] = H(s, i, k);
    for (int i = 0; i <= 4; i++) g5[i] = G(s, i, k);
}

/* ---------------------------------------------------------------- collision (eq. 6-17) */
static double nu_of(const or_params* P) { return (2.0 * P->tau_f - 1.0) / 6.0; }   /* eq. 10 */

static void collide_node(const or_state* s, int porous, const double* h8, const double* g5,
                         double* h8s, double* g5s)
{
    const or_params* P = &s->P;
    moments m = moments_of(s, h8, g5);

    /* eq. 15-16: buoyancy with the constant part absorbed into p */
    double Bx = P->gbeta * (m.T - P->T0) * s->gx_hat;
    double By = P->gbeta * (m.T - P->T0) * s->gy_hat;
    double Dx = 0.0, Dy = 0.0;
    if (porous) {
        /* eq. 4 as a body force: Darcy drag on the mid-step velocity
         * u_D = u + (F_b + F_D)/2 with F_D = -(nu/K) u_D, solved for u_D */
        double nuK = nu_of(P) / P->K;
        double uDx = (m.ux + 0.5 * Bx) / (1.0 + 0.5 * nuK);
        double uDy = (m.uy + 0.5 * By) / (1.0 + 0.5 * nuK);
        Dx = -nuK * uDx;
        Dy = -nuK * uDy;
    }

    double omega = 1.0 / P->tau_f;
    for (int i = 1; i <= 8; i++) {
        double heq = lambda_i(i) * m.dp + S(i, m.ux, m.uy);                 /* eq. 7 */
        /* eq. 17: buoyancy on the axis links only */
        double Fi = (i <= 4) ? 0.5 * (ex[i] * Bx + ey[i] * By) : 0.0;
        /* Darcy drag on all links with weights 3 w_i, which matches the linear term of
         * eq. 8 (zero mass, momentum F_D, zero second moment, third moment F_D/3); the
         * axis-only form is unstable once nu/K exceeds about 4 */
        Fi += 3.0 * w_flow(i) * (ex[i] * Dx + ey[i] * Dy);
        h8s[i - 1] = h8[i - 1] - omega * (h8[i - 1] - heq) + Fi;           /* eq. 6 */
    }

    double omegaT = 1.0 / P->tau_t;
    double cs2T = (1.0 - P->w0) / 2.0;
    for (int i = 0; i <= 4; i++) {
        double eu = ex[i] * m.ux + ey[i] * m.uy;
        double geq = w_heat(P, i) * ((m.T - P->T_ref) + m.T * eu / cs2T);  /* eq. 12 */
        g5s[i] = g5[i] - omegaT * (g5[i] - geq);                            /* eq. 11 */
    }
}

/* ---------------------------------------------------------------- boundaries */
/* eq. 4 over the meshwork thickness: u = (K/mu) (p_IOP - p_sc) / h_TM, mu = nu at unit density */
static double seepage_speed(const or_params* P, double p_iop)
{
    return P->K_tm / nu_of(P) * ((p_iop - P->p_sc) / P->h_tm);
}

static double wall_temperature(const or_state* s, int wall)
{
    return wall == OR_WALL_CORNEA ? s->P.T_cornea : s->P.T_iris;
}

/* Deviation-form equilibria (eq. 7-8, eq. 12) and post-collision moments, for the paper's
 * boundary scheme. */
static double heq_of(int i, double dp, double ux, double uy) { return lambda_i(i) * dp + S(i, ux, uy); }

static double geq_of(const or_params* P, int i, double T, double ux, double uy)
{
    double eu = ex[i] * ux + ey[i] * uy;
    return w_heat(P, i) * ((T - P->T_ref) + T * eu / ((1.0 - P->w0) / 2.0));
}

/* moments of node k's post-collision populations: (p* - p_ref, u*, T*) */
static moments post_moments(const or_state* s, size_t k)
{
    double h8[8], g5[5];
    for (int i = 1; i <= 8; i++) h8[i - 1] = s->hs[(size_t)(i - 1) * s->n + k];
    for (int i = 0; i <= 4; i++) g5[i] = s->gs[(size_t)i * s->n + k];
    return moments_of(s, h8, g5);
}

/* One full time step. */
static void step_once(or_state* s)
{
    const or_params* P = &s->P;
    size_t n = s->n;

    /* (1) collide every active node into hs/gs */
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; k++) {
        if (!is_active(s, k)) continue;
        double h8[8], g5[5], h8s[8], g5s[5];
        gather(s, k, h8, g5);
        collide_node(s, s->cls[k] == OR_POROUS, h8, g5, h8s, g5s);
        for (int i = 1; i <= 8; i++) s->hs[(size_t)(i - 1) * n + k] = h8s[i - 1];
        for (int i = 0; i <= 4; i++) s->gs[(size_t)i * n + k] = g5s[i];
    }

    /* (2) stream: poison the targets so an unwritten slot shows as NaN */
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < 8 * n; k++) s->hn[k] = NAN;
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < 5 * n; k++) s->gn[k] = NAN;

    double q_out = 0.0, q_in = 0.0;
    /* every (target node, direction) slot has exactly one writer, so rows are independent */
#pragma omp parallel for schedule(static) reduction(+ : q_out, q_in)
    for (int y = 0; y < s->ny; y++) {
        for (int x = 0; x < s->nx; x++) {
            size_t k = (size_t)y * s->nx + x;
            if (!is_active(s, k)) continue;
            for (int i = 1; i <= 8; i++) {
                double hout = s->hs[(size_t)(i - 1) * n + k];
                long kk = neighbour(s, x, y, ex[i], ey[i]);
                int c = kk < 0 ? OR_SOLID : s->cls[kk];
                int ib = opposite[i];
                double* back = &s->hn[(size_t)(ib - 1) * n + k];
                if (c == OR_FLUID || c == OR_POROUS) {
                    s->hn[(size_t)(i - 1) * n + kk] = hout;
                } else if (c == OR_SOLID) {
                    double q = -1.0;
                    if (P->bc_scheme == OR_BC_PAPER && s->wall_of[k] >= 0)
                        q = s->wall_q[(size_t)s->wall_of[k] * 8 + (i - 1)];
                    long kb = neighbour(s, x, y, -ex[i], -ey[i]);       /* x - e_o */
                    if (q >= 0.5) {                                     /* interpolated bounce-back */
                        *back = hout / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * s->hs[(size_t)(ib - 1) * n + k];
                    } else if (q > 0.0 && kb >= 0 && is_active(s, (size_t)kb)) {
                        *back = 2.0 * q * hout + (1.0 - 2.0 * q) * s->hs[(size_t)(i - 1) * n + kb];
                    } else {
                        *back = hout;                                   /* half-way bounce-back */
                    }
                } else if (P->bc_scheme == OR_BC_PAPER) {                /* INLET or OUTLET, extrapolation */
                    moments ms = post_moments(s, k);
                    double dpb = ms.dp, uxb = ms.ux, uyb = ms.uy;
                    if (c == OR_INLET) {
                        uxb = P->u_in_x;
                        uyb = P->u_in_y;
                    } else if (P->outlet_mode == OR_OUTLET_LUMPED) {
                        int d = s->wall[kk] + 1;
                        uxb = ex[d] * s->u_seep;
                        uyb = ey[d] * s->u_seep;
                    } else {
                        dpb = P->p_out - P->p_ref;
                    }
                    *back = heq_of(ib, dpb, uxb, uyb) + (s->hs[(size_t)(ib - 1) * n + k] - heq_of(ib, ms.dp, ms.ux, ms.uy));
                    if (c == OR_INLET) q_in += *back - hout;
                    else q_out += hout - *back;
                } else if (c == OR_INLET) {
                    double eu = ex[i] * P->u_in_x + ey[i] * P->u_in_y;
                    *back = hout - 6.0 * w_flow(i) * eu;                /* moving wall u_in */
                    q_in += *back - hout;
                } else if (P->outlet_mode == OR_OUTLET_LUMPED) { /* OR_OUTLET, lumped meshwork */
                    int d = s->wall[kk] + 1;                            /* outward axis link */
                    double eu = (ex[i] * ex[d] + ey[i] * ey[d]) * s->u_seep;
                    *back = hout - 6.0 * w_flow(i) * eu;                /* moving wall u_s n */
                    q_out += hout - *back;
                } else { /* OR_OUTLET */
                    *back = -hout + 2.0 * lambda_i(i) * (P->p_out - P->p_ref); /* pressure ABB */
                    q_out += hout - *back;
                }
            }
            for (int i = 1; i <= 4; i++) {
                double gout = s->gs[(size_t)i * n + k];
                long kk = neighbour(s, x, y, ex[i], ey[i]);
                int c = kk < 0 ? OR_SOLID : s->cls[kk];
                int wall = kk < 0 ? OR_WALL_BOX : s->wall[kk];
                int ib = opposite[i];
                double* back = &s->gn[(size_t)ib * n + k];
                if (c == OR_FLUID || c == OR_POROUS) {
                    s->gn[(size_t)i * n + kk] = gout;
                } else if (((c == OR_SOLID && wall != OR_WALL_BOX) || c == OR_INLET) && P->bc_scheme == OR_BC_PAPER) {
                    double Tw = (c == OR_INLET) ? P->T_inlet : wall_temperature(s, wall);
                    double uxb = c == OR_INLET ? P->u_in_x : 0.0, uyb = c == OR_INLET ? P->u_in_y : 0.0;
                    moments ms = post_moments(s, k);                        /* extrapolation */
                    *back = geq_of(P, ib, Tw, uxb, uyb) + (s->gs[(size_t)ib * n + k] - geq_of(P, ib, ms.T, ms.ux, ms.uy));
                } else if ((c == OR_SOLID && wall != OR_WALL_BOX) || c == OR_INLET) {
                    double Tw = (c == OR_INLET) ? P->T_inlet : wall_temperature(s, wall);
                    *back = -gout + 2.0 * w_heat(P, i) * (Tw - P->T_ref);   /* Dirichlet ABB */
                } else {
                    *back = gout;                                           /* adiabatic */
                }
            }
            s->gn[k] = s->gs[k];   /* rest population stays */
        }
    }
    s->q_out_last = q_out;
    s->q_in_last = q_in;

    /* (3) swap */
    double* t = s->h; s->h = s->hn; s->hn = t;
    t = s->g; s->g = s->gn; s->gn = t;
    s->step++;
}

/* ---------------------------------------------------------------- observables */
static void observe(or_state* s)
{
    const or_params* P = &s->P;
    double sum_dp = 0.0, cnt = 0.0, du2 = 0.0, u2 = 0.0, dT2 = 0.0, T2 = 0.0;
    double mf = 0.0, mt = 0.0, umax = 0.0;
    int64_t bad = 0;
    for (size_t k = 0; k < s->n; k++) {
        if (!is_active(s, k)) continue;
        double h8[8], g5[5];
        gather(s, k, h8, g5);
        moments m = moments_of(s, h8, g5);
        if (!isfinite(m.dp) || !isfinite(m.ux) || !isfinite(m.uy) || !isfinite(m.T)) bad++;
        if (s->cls[k] == OR_FLUID) { sum_dp += m.dp; cnt += 1.0; }
        double dx = m.ux - s->u_prev_x[k], dy = m.uy - s->u_prev_y[k];
        du2 += dx * dx + dy * dy;
        u2 += m.ux * m.ux + m.uy * m.uy;
        double dT = m.T - s->T_prev[k];
        dT2 += dT * dT;
        T2 += (m.T - P->T_ref) * (m.T - P->T_ref);
        double um = sqrt(m.ux * m.ux + m.uy * m.uy);
        if (um > umax) umax = um;
        for (int i = 0; i < 8; i++) mf += h8[i];
        for (int i = 0; i < 5; i++) mt += g5[i];
        s->u_prev_x[k] = m.ux;
        s->u_prev_y[k] = m.uy;
        s->T_prev[k] = m.T;
    }

    /* wall shear stress from the non-equilibrium stress, sigma = -(1 - 1/(2 tau)) Pi^neq */
    double ws[3] = {0, 0, 0}, wm[3] = {0, 0, 0}, wc[3] = {0, 0, 0};
    for (int w = 0; w < s->n_walls; w++) {
        size_t k = (size_t)s->wall_node[w];
        double h8[8], g5[5];
        gather(s, k, h8, g5);
        moments m = moments_of(s, h8, g5);
        double pxx = 0.0, pxy = 0.0, pyy = 0.0;
        for (int i = 1; i <= 8; i++) {
            double neq = h8[i - 1] - (lambda_i(i) * m.dp + S(i, m.ux, m.uy));
            pxx += ex[i] * ex[i] * neq;
            pxy += ex[i] * ey[i] * neq;
            pyy += ey[i] * ey[i] * neq;
        }
        double f = -(1.0 - 0.5 / P->tau_f);
        double sxx = f * pxx, sxy = f * pxy, syy = f * pyy;
        double nx_ = s->wall_nx[w], ny_ = s->wall_ny[w];
        double tx = sxx * nx_ + sxy * ny_, ty = sxy * nx_ + syy * ny_;
        double tn = tx * nx_ + ty * ny_;
        double tau_w = sqrt((tx - tn * nx_) * (tx - tn * nx_) + (ty - tn * ny_) * (ty - tn * ny_));
        int id = s->wall_id[w];
        if (id < 1 || id > 2) continue;
        ws[id] += tau_w;
        wc[id] += 1.0;
        if (tau_w > wm[id]) wm[id] = tau_w;
    }

    double D = (double)P->check_interval;
    or_observables* o = &s->obs;
    o->step = s->step;
    o->p_mean_fluid = P->p_ref + (cnt > 0 ? sum_dp / cnt : 0.0);
    o->iop_gauge = o->p_mean_fluid - P->p_out;
    o->q_in = s->q_in_last;
    o->q_out = s->q_out_last;
    o->wss_cornea_mean = wc[1] > 0 ? ws[1] / wc[1] : 0.0;
    o->wss_cornea_max = wm[1];
    o->wss_iris_mean = wc[2] > 0 ? ws[2] / wc[2] : 0.0;
    o->wss_iris_max = wm[2];
    o->resid_u = u2 > 0 ? sqrt(du2) / (D * sqrt(u2)) : sqrt(du2) / D;
    o->resid_T = T2 > 0 ? sqrt(dT2) / (D * sqrt(T2)) : sqrt(dT2) / D;
    o->u_max = umax;
    o->mass_flow = mf;
    o->mass_thermal = mt;
    o->n_nonfinite = bad;
    /* lumped meshwork: Darcy seepage from the pressure drop across it, for the next interval */
    if (P->outlet_mode == OR_OUTLET_LUMPED)
        s->u_seep = seepage_speed(P, o->p_mean_fluid);
    o->u_seep = s->u_seep;
}

static void set_prev_from_state(or_state* s)
{
    for (size_t k = 0; k < s->n; k++) {
        if (!is_active(s, k)) { s->u_prev_x[k] = s->u_prev_y[k] = s->T_prev[k] = 0.0; continue; }
        double h8[8], g5[5];
        gather(s, k, h8, g5);
        moments m = moments_of(s, h8, g5);
        s->u_prev_x[k] = m.ux;
        s->u_prev_y[k] = m.uy;
        s->T_prev[k] = m.T;
    }
}

/* The paper's scheme at t = 0: the populations entering from INLET / OUTLET nodes and
 * Dirichlet thermal walls are what the extrapolation gives when every post-collision
 * population is the initial equilibrium. */
static void initial_boundary_populations(or_state* s)
{
    const or_params* P = &s->P;
    size_t n = s->n;
    memcpy(s->hs, s->h, 8 * n * sizeof(double));
    memcpy(s->gs, s->g, 5 * n * sizeof(double));
    for (int y = 0; y < s->ny; y++)
        for (int x = 0; x < s->nx; x++) {
            size_t k = (size_t)y * s->nx + x;
            if (!is_active(s, k)) continue;
            moments ms = post_moments(s, k);
            for (int i = 1; i <= 8; i++) {
                long kk = neighbour(s, x, y, ex[i], ey[i]);
                int c = kk < 0 ? OR_SOLID : s->cls[kk];
                int ib = opposite[i];
                if (c == OR_INLET || c == OR_OUTLET) {
                    double dpb = ms.dp, uxb = ms.ux, uyb = ms.uy;
                    if (c == OR_INLET) {
                        uxb = P->u_in_x;
                        uyb = P->u_in_y;
                    } else if (P->outlet_mode == OR_OUTLET_LUMPED) {
                        int d = s->wall[kk] + 1;
                        uxb = ex[d] * s->u_seep;
                        uyb = ey[d] * s->u_seep;
                    } else {
                        dpb = P->p_out - P->p_ref;
                    }
                    H(s, ib, k) = heq_of(ib, dpb, uxb, uyb) + (s->hs[(size_t)(ib - 1) * n + k] - heq_of(ib, ms.dp, ms.ux, ms.uy));
                }
                if (i > 4) continue;
                int wall = kk < 0 ? OR_WALL_BOX : s->wall[kk];
                if ((c == OR_SOLID && wall != OR_WALL_BOX) || c == OR_INLET) {
                    double Tw = (c == OR_INLET) ? P->T_inlet : wall_temperature(s, wall);
                    double uxb = c == OR_INLET ? P->u_in_x : 0.0, uyb = c == OR_INLET ? P->u_in_y : 0.0;
                    G(s, ib, k) = geq_of(P, ib, Tw, uxb, uyb) + (s->gs[(size_t)ib * n + k] - geq_of(P, ib, ms.T, ms.ux, ms.uy));
                }
            }
        }
}

/* ---------------------------------------------------------------- API */
or_state* or_create(const or_params* P, const uint8_t* mask, int n_walls, const int32_t* wall_node,
                    const int32_t* wall_id, const double* wall_nx, const double* wall_ny, const double* wall_q)
{
    if (P->nx < 3 || P->ny < 3 || P->tau_f <= 0.5 || P->tau_t <= 0.5 || P->check_interval < 1) return NULL;
    if (P->outlet_mode == OR_OUTLET_LUMPED && !(P->K_tm > 0 && P->h_tm > 0)) return NULL;
    or_state* s = (or_state*)calloc(1, sizeof(or_state));
    s->P = *P;
    s->gx_hat = sin(P->gravity_angle);
    s->gy_hat = cos(P->gravity_angle);
    s->nx = P->nx;
    s->ny = P->ny;
    s->n = (size_t)P->nx * P->ny;
    size_t n = s->n;
    s->cls = (uint8_t*)malloc(n);
    s->wall = (uint8_t*)malloc(n);
    for (size_t k = 0; k < n; k++) {
        s->cls[k] = mask[k] & 7;
        s->wall[k] = (mask[k] >> 3) & 3;
    }
    s->h = (double*)malloc(8 * n * sizeof(double));
    s->hs = (double*)malloc(8 * n * sizeof(double));
    s->hn = (double*)malloc(8 * n * sizeof(double));
    s->g = (double*)malloc(5 * n * sizeof(double));
    s->gs = (double*)malloc(5 * n * sizeof(double));
    s->gn = (double*)malloc(5 * n * sizeof(double));
    s->u_prev_x = (double*)calloc(n, sizeof(double));
    s->u_prev_y = (double*)calloc(n, sizeof(double));
    s->T_prev = (double*)calloc(n, sizeof(double));
    s->n_walls = n_walls;
    s->wall_node = (int32_t*)malloc((n_walls + 1) * sizeof(int32_t));
    s->wall_id = (int32_t*)malloc((n_walls + 1) * sizeof(int32_t));
    s->wall_nx = (double*)malloc((n_walls + 1) * sizeof(double));
    s->wall_ny = (double*)malloc((n_walls + 1) * sizeof(double));
    s->wall_q = (double*)malloc(((size_t)n_walls + 1) * 8 * sizeof(double));
    s->wall_of = (int32_t*)malloc(n * sizeof(int32_t));
    for (size_t k = 0; k < n; k++) s->wall_of[k] = -1;
    for (int w = 0; w < n_walls; w++) {
        s->wall_node[w] = wall_node[w];
        s->wall_id[w] = wall_id[w];
        s->wall_nx[w] = wall_nx[w];
        s->wall_ny[w] = wall_ny[w];
        for (int i = 0; i < 8; i++) s->wall_q[(size_t)w * 8 + i] = wall_q ? wall_q[(size_t)w * 8 + i] : -1.0;
        s->wall_of[wall_node[w]] = w;
    }

    /* initial state: equilibrium at (p_init, u = 0, T_init), eq. 7 and eq. 12 */
    for (size_t k = 0; k < n; k++) {
        int act = is_active(s, k);
        for (int i = 1; i <= 8; i++)
            H(s, i, k) = act ? lambda_i(i) * (P->p_init - P->p_ref) + S(i, 0.0, 0.0) : NAN;
        for (int i = 0; i <= 4; i++)
            G(s, i, k) = act ? w_heat(P, i) * (P->T_init - P->T_ref) : NAN;
    }
    s->u_seep = P->outlet_mode == OR_OUTLET_LUMPED ? seepage_speed(P, P->p_init) : 0.0;
    if (P->bc_scheme == OR_BC_PAPER) initial_boundary_populations(s);
    set_prev_from_state(s);
    memset(&s->obs, 0, sizeof(s->obs));
    return s;
}

void or_destroy(or_state* s)
{
    if (!s) return;
    free(s->cls); free(s->wall);
    free(s->h); free(s->hs); free(s->hn);
    free(s->g); free(s->gs); free(s->gn);
    free(s->u_prev_x); free(s->u_prev_y); free(s->T_prev);
    free(s->wall_node); free(s->wall_id); free(s->wall_nx); free(s->wall_ny);
    free(s->wall_q); free(s->wall_of);
    free(s);
}

void or_step(or_state* s, int64_t nsteps)
{
    for (int64_t t = 0; t < nsteps; t++) {
        step_once(s);
        if (s->step % s->P.check_interval == 0) observe(s);
    }
}

int64_t or_step_count(const or_state* s) { return s->step; }

/* Replace the lumped meshwork's K_TM, h_TM and p_sc (the thickness calibration of section
 * 3.1).  The seepage speed in effect becomes that of the new values at the IOP of the last
 * check step (p_init before the first one). */
void or_set_outlet(or_state* s, double K_tm, double h_tm, double p_sc)
{
    s->P.K_tm = K_tm;
    s->P.h_tm = h_tm;
    s->P.p_sc = p_sc;
    s->u_seep = seepage_speed(&s->P, s->obs.step > 0 ? s->obs.p_mean_fluid : s->P.p_init);
}

void or_observables_get(const or_state* s, or_observables* out) { *out = s->obs; }

void or_observe(or_state* s, or_observables* out)
{
    observe(s);
    *out = s->obs;
}

/* Macroscopic fields of the current (pre-collision) state; NaN at non-active nodes. */
void or_fields(const or_state* s, double* dp, double* ux, double* uy, double* T)
{
    for (size_t k = 0; k < s->n; k++) {
        if (!is_active(s, k)) { dp[k] = ux[k] = uy[k] = T[k] = NAN; continue; }
        double h8[8], g5[5];
        gather(s, k, h8, g5);
        moments m = moments_of(s, h8, g5);
        dp[k] = m.dp;
        ux[k] = m.ux;
        uy[k] = m.uy;
        T[k] = m.T;
    }
}

void or_get_populations(const or_state* s, double* h, double* g)
{
    memcpy(h, s->h, 8 * s->n * sizeof(double));
    memcpy(g, s->g, 5 * s->n * sizeof(double));
}

/* Replace the pre-collision state; values at non-active nodes are ignored (kept NaN). */
void or_set_populations(or_state* s, const double* h, const double* g)
{
    for (size_t k = 0; k < s->n; k++) {
        int act = is_active(s, k);
        for (int q = 0; q < 8; q++) s->h[(size_t)q * s->n + k] = act ? h[(size_t)q * s->n + k] : NAN;
        for (int q = 0; q < 5; q++) s->g[(size_t)q * s->n + k] = act ? g[(size_t)q * s->n + k] : NAN;
    }
    set_prev_from_state(s);
}

/* Single-node collision on caller-given populations (for unit checks). */
void or_collide_node(const or_params* P, int porous, const double* h8, const double* g5,
                     double* h8s, double* g5s)
{
    or_state s;
    memset(&s, 0, sizeof(s));
    s.P = *P;
    s.gx_hat = sin(P->gravity_angle);
    s.gy_hat = cos(P->gravity_angle);
    collide_node(&s, porous, h8, g5, h8s, g5s);
}

/* Equilibrium populations (deviation form) for given (p, u, T). */
void or_equilibrium(const or_params* P, double p, double ux, double uy, double T, double* h8, double* g5)
{
    double cs2T = (1.0 - P->w0) / 2.0;
    for (int i = 1; i <= 8; i++) h8[i - 1] = lambda_i(i) * (p - P->p_ref) + S(i, ux, uy);
    for (int i = 0; i <= 4; i++) {
        double eu = ex[i] * ux + ey[i] * uy;
        g5[i] = w_heat(P, i) * ((T - P->T_ref) + T * eu / cs2T);
    }
}

void or_moments(const or_params* P, const double* h8, const double* g5, double* out4)
{
    or_state s;
    memset(&s, 0, sizeof(s));
    s.P = *P;
    moments m = moments_of(&s, h8, g5);
    out4[0] = m.dp;
    out4[1] = m.ux;
    out4[2] = m.uy;
    out4[3] = m.T;
}
