/*
 * Plain FP64 CPU oracle of one coupled time step of the conservative
 * Allen-Cahn phase-field lattice Boltzmann method (D3Q15, SRT) and the
 * velocity-based hydrodynamic lattice Boltzmann method (D3Q27, weighted
 * orthogonal MRT) of Holzer, Bauer, Koestler and Ruede (IJHPCA 2020,
 * arXiv 2012.06144), Sections 3.1 and 3.2.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, literal checker the
 * GPU library is compared against.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What follows each formula of the paper in its own words and order:
 *   - lattice weights: the standard D3Q15 / D3Q27 sets (not printed in the
 *     paper; pinned by the isotropy conditions in the tests);
 *   - phase-field step: pull streaming, phi = sum of the pulled PDFs
 *     (eq. updatePhaseField), isotropic gradient (eq. grad), normal and
 *     theta (eq. allen_cahn), forcing F^phi (eq. interfaceTracking),
 *     equilibrium phi*Gamma, single-relaxation collision (eq. lb_interface
 *     with a scalar relaxation rate, as used in Section 5);
 *   - hydrodynamic step: moments, rho and tau interpolation (eq. density
 *     and the tau interpolation of Section 3.2), isotropic gradient and
 *     Laplacian (eqs. grad, lap), chemical potential (eq. chemPot),
 *     pressure, surface tension, viscous and body forces (eqs.
 *     forceHydro, pressure_force, surfaceTension, viscousForce, and the
 *     buoyancy of Section 6.1), velocity update (eq. updateVelocityField),
 *     and the moment-space collision m* = m - S(m - m_eq + F_m/2) + F_m,
 *     g* = M^-1 m* (eq. improved_collision and the listing beside it),
 *     with a literal 27x27 moment matrix; push streaming.
 *
 * Readings where the paper is silent or ambiguous (each also listed in
 * the design notes of the repository):
 *   - the phase relaxation rate is 1/(tau_phi + 1/2) with tau_phi = M/cs^2
 *     (the literal 1/tau_phi is outside the stable range);
 *   - the hydrodynamic tau is the model tau of nu = tau*cs^2, rate
 *     s_nu = 1/(tau + 1/2) on all six second-order moments, 1 elsewhere;
 *   - the moment basis is Gram-Schmidt of the 27 monomials x^a y^b z^c
 *     (a,b,c <= 2) in total-degree order under sum_i w_i f_i g_i, rows not
 *     normalised (rows 1..3 stay e_x, e_y, e_z, so F_m = (0, F/rho, 0..));
 *   - fused time levels: the phase step takes grad(phi) and theta from the
 *     previous phi field (phi_A) and u from the previous hydrodynamic step;
 *     the hydrodynamic step takes the new phi (phi_B) and uses the stored
 *     (old) u only inside the viscous force;
 *   - the normal is grad/(|grad| + eps); gradients are summed as
 *     antisymmetric pair differences so an exactly symmetric field gives an
 *     exactly zero gradient;
 *   - rho and tau interpolations divide by (phi_H - phi_L);
 *   - y walls: rows 0 and ny-1 are solid, halfway bounce-back for h and g,
 *     phi stencils mirror the wall row onto the first fluid row;
 *   - buoyancy F_b = (rho - rho_ref) a: rho_ref = 0 is the printed rho g;
 *     rho_ref = rho_H leaves out the hydrostatic pressure of the heavy fluid
 *     (a uniform force the walls balance).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q15 15
#define Q19 19
#define Q27 27
#define QMAX 27

typedef struct {
    int32_t nx, ny, nz;
    int32_t walls_y;
    double phi_L, phi_H, xi, mobility, sigma;
    double rho_L, rho_H, tau_L, tau_H;
    double accel[3];
    double rho_ref;      /* buoyancy reference density: F_b = (rho - rho_ref) a */
    double normal_eps;
    int32_t density_literal; /* 1: eq. density for every phi (no clamp) */
    int32_t lattice_phase;   /* velocity set of the phase-field step: 15 (0 = 15), 19 or 27 */
    int32_t lattice_hydro;   /* velocity set of the hydrodynamic step: 27 (0 = 27), 19 or 15 */
    int32_t phase_mrt;       /* 1: raw-moment MRT phase-field collision instead of SRT */
} orc_params;

typedef struct {
    double mass;
    double momentum[3];
    double gas_volume;
    double centroid[3];
    double rise_velocity;
    double interface_sum;   /* sum 4 chi (1 - chi) */
    double grad_sum;        /* sum |grad phi| / (phi_H - phi_L) */
    double xi_eff;
    double max_speed;
} orc_stats;

/* ---- velocity sets ------------------------------------------------------
 * Canonical order: rest, then axis pairs, then (D3Q27) edge pairs, then
 * corner pairs; every odd index i has its opposite at i+1.               */
static const int E15[Q15][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

static const int E27[Q27][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

/* D3Q19: rest, axis pairs and edge pairs (the first 19 vectors of D3Q27). */
static const int E19[Q19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double W15[Q15];
static double W19[Q19];
static double W27[Q27];

typedef struct {
    int q;
    const int (*e)[3];
    const double *w;
} orc_lat;

static void init_weights(void)
{
    for (int i = 0; i < Q15; ++i) {
        int n = abs(E15[i][0]) + abs(E15[i][1]) + abs(E15[i][2]);
        W15[i] = (n == 0) ? 2.0 / 9.0 : (n == 1) ? 1.0 / 9.0 : 1.0 / 72.0;
    }
    for (int i = 0; i < Q19; ++i) {
        int n = abs(E19[i][0]) + abs(E19[i][1]) + abs(E19[i][2]);
        W19[i] = (n == 0) ? 1.0 / 3.0 : (n == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
    }
    for (int i = 0; i < Q27; ++i) {
        int n = abs(E27[i][0]) + abs(E27[i][1]) + abs(E27[i][2]);
        W27[i] = (n == 0) ? 8.0 / 27.0 : (n == 1) ? 2.0 / 27.0
               : (n == 2) ? 1.0 / 54.0 : 1.0 / 216.0;
    }
}

/* Velocity set of q directions (15, 19 or 27; anything else gives D3Q27). */
static orc_lat lat_of(int q)
{
    orc_lat L;
    L.q = q == Q15 ? Q15 : (q == Q19 ? Q19 : Q27);
    L.e = q == Q15 ? E15 : (q == Q19 ? E19 : E27);
    L.w = q == Q15 ? W15 : (q == Q19 ? W19 : W27);
    return L;
}

static int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

static const double CS2 = 1.0 / 3.0; /* c_s^2 with dx = dt = 1 */

/* ---- lattice queries used by the pins ---------------------------------- */
int orc_velocity_set(int32_t q, int32_t *e, double *w)
{
    init_weights();
    if (q != Q15 && q != Q19 && q != Q27) return -1;
    const orc_lat L = lat_of(q);
    for (int i = 0; i < L.q; ++i) {
        for (int a = 0; a < 3; ++a) e[3 * i + a] = L.e[i][a];
        w[i] = L.w[i];
    }
    return 0;
}

/* Gamma_i(u) = w_i [1 + e.u/cs^2 + (e.u)^2/(2 cs^4) - u.u/(2 cs^2)]
 * (dimensionless distribution of Section 3.1).                          */
static double gamma_i(const int e[3], double w, const double u[3])
{
    double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return w * (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

void orc_gamma(int32_t q, const double *u, double *out)
{
    init_weights();
    const orc_lat L = lat_of(q);
    for (int i = 0; i < L.q; ++i) out[i] = gamma_i(L.e[i], L.w[i], u);
}

/* g_eq_i = p* w_i + (Gamma_i - w_i)  (Section 3.2) */
static void hydro_equilibrium(orc_lat L, double pstar, const double u[3], double *out)
{
    for (int i = 0; i < L.q; ++i)
        out[i] = pstar * L.w[i] + (gamma_i(L.e[i], L.w[i], u) - L.w[i]);
}

void orc_hydro_equilibrium(double pstar, const double *u, double *out)
{
    init_weights();
    hydro_equilibrium(lat_of(Q27), pstar, u, out);
}

/* F^phi_i = theta w_i e_i . n  (eq. interfaceTracking, dt = 1) */
static void phase_forcing(orc_lat L, double theta, const double n[3], double *out)
{
    for (int i = 0; i < L.q; ++i)
        out[i] = theta * L.w[i] * (L.e[i][0] * n[0] + L.e[i][1] * n[1] + L.e[i][2] * n[2]);
}

void orc_phase_forcing(double theta, const double *n, double *out)
{
    init_weights();
    phase_forcing(lat_of(Q15), theta, n, out);
}

/* ---- weighted-orthogonal moment matrices -------------------------------------
 * For a velocity set of q directions: the monomials x^a y^b z^c (a, b, c in
 * {0, 1, 2}) in order of total degree, orthogonalised one after another
 * (modified Gram-Schmidt under sum_i w_i f_i g_i, no normalisation); a
 * monomial that is a combination of the earlier ones on this set (its
 * remainder vanishes) is left out, which leaves exactly q rows.  The raw
 * moment matrix of the phase-field MRT takes the same monomials without
 * the orthogonalisation.                                                   */
typedef struct {
    int ready;
    int q;
    double M[QMAX][QMAX];    /* row k: orthogonalised monomial k at e_i */
    double Minv[QMAX][QMAX];
    double R[QMAX][QMAX];    /* row k: the raw monomial k at e_i */
    double Rinv[QMAX][QMAX];
    int deg[QMAX];           /* total degree of the monomial of row k */
    int expo[QMAX][3];       /* exponents (a, b, c) of the monomial of row k */
} orc_mrt;
static orc_mrt MRT[3];       /* D3Q15, D3Q19, D3Q27 */

static int mrt_slot(int q) { return q == Q15 ? 0 : (q == Q19 ? 1 : 2); }

static double monomial(const int e[3], int a, int b, int c)
{
    double v = 1.0;
    for (int k = 0; k < a; ++k) v *= e[0];
    for (int k = 0; k < b; ++k) v *= e[1];
    for (int k = 0; k < c; ++k) v *= e[2];
    return v;
}

static double winner(orc_lat L, const double *f, const double *g)
{
    double s = 0.0;
    for (int i = 0; i < L.q; ++i) s += L.w[i] * f[i] * g[i];
    return s;
}

/* Gauss-Jordan inverse of an n x n matrix with partial pivoting. */
static int invert_n(int n, double A[QMAX][QMAX], double R[QMAX][QMAX])
{
    double T[QMAX][2 * QMAX];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            T[r][c] = (c < n) ? A[r][c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(T[r][col]) > fabs(T[piv][col])) piv = r;
        if (fabs(T[piv][col]) < 1e-14) return -1;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = T[col][c]; T[col][c] = T[piv][c]; T[piv][c] = t;
            }
        double d = T[col][col];
        for (int c = 0; c < 2 * n; ++c) T[col][c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = T[r][col];
            if (f != 0.0)
                for (int c = 0; c < 2 * n; ++c) T[r][c] -= f * T[col][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) R[r][c] = T[r][n + c];
    return 0;
}

static orc_mrt *build_mrt_q(int q)
{
    orc_mrt *m = &MRT[mrt_slot(q)];
    if (m->ready) return m;
    init_weights();
    const orc_lat L = lat_of(q);
    m->q = L.q;
    int k = 0;
    for (int deg = 0; deg <= 6 && k < L.q; ++deg)
        for (int a = 2; a >= 0; --a)
            for (int b = 2; b >= 0; --b)
                for (int c = 2; c >= 0; --c) {
                    if (a + b + c != deg || k >= L.q) continue;
                    double row[QMAX], raw[QMAX];
                    for (int i = 0; i < L.q; ++i) raw[i] = row[i] = monomial(L.e[i], a, b, c);
                    for (int s2 = 0; s2 < k; ++s2) {
                        double proj = winner(L, row, m->M[s2]) / winner(L, m->M[s2], m->M[s2]);
                        for (int i = 0; i < L.q; ++i) row[i] -= proj * m->M[s2][i];
                    }
                    if (winner(L, row, row) < 1e-12) continue;  /* dependent on this set */
                    for (int i = 0; i < L.q; ++i) {
                        m->M[k][i] = row[i];
                        m->R[k][i] = raw[i];
                    }
                    m->deg[k] = deg;
                    m->expo[k][0] = a;
                    m->expo[k][1] = b;
                    m->expo[k][2] = c;
                    ++k;
                }
    if (k != L.q) return NULL;
    if (invert_n(L.q, m->M, m->Minv) != 0) return NULL;
    if (invert_n(L.q, m->R, m->Rinv) != 0) return NULL;
    m->ready = 1;
    return m;
}

static int build_mrt(void) { return build_mrt_q(Q27) ? 0 : -1; }

/* Export M, M^-1 and the degree of each row for the pins (D3Q27). */
int orc_moment_matrix(double *M, double *Minv, int32_t *deg)
{
    const orc_mrt *m = build_mrt_q(Q27);
    if (!m) return -1;
    for (int r = 0; r < Q27; ++r) {
        deg[r] = m->deg[r];
        for (int c = 0; c < Q27; ++c) {
            M[r * Q27 + c] = m->M[r][c];
            Minv[r * Q27 + c] = m->Minv[r][c];
        }
    }
    return 0;
}

/* The same for a velocity set of q directions, with the raw monomial
 * matrix and its inverse and the exponents of each row.                  */
int orc_moment_matrix_q(int32_t q, double *M, double *Minv, double *R, double *Rinv, int32_t *deg,
                        int32_t *expo)
{
    if (q != Q15 && q != Q19 && q != Q27) return -1;
    const orc_mrt *m = build_mrt_q(q);
    if (!m) return -1;
    for (int r = 0; r < q; ++r) {
        deg[r] = m->deg[r];
        for (int a = 0; a < 3; ++a) expo[3 * r + a] = m->expo[r][a];
        for (int c = 0; c < q; ++c) {
            M[r * q + c] = m->M[r][c];
            Minv[r * q + c] = m->Minv[r][c];
            R[r * q + c] = m->R[r][c];
            Rinv[r * q + c] = m->Rinv[r][c];
        }
    }
    return 0;
}

static void relaxation_rates(const orc_mrt *m, double s_nu, double *S)
{
    for (int k = 0; k < m->q; ++k) S[k] = (m->deg[k] == 2) ? s_nu : 1.0;
}

static void matvec(const orc_mrt *m, const double A[QMAX][QMAX], const double *x, double *y)
{
    for (int r = 0; r < m->q; ++r) {
        double s = 0.0;
        for (int c = 0; c < m->q; ++c) s += A[r][c] * x[c];
        y[r] = s;
    }
}

/* Sum_k e_k e_k^T (Omega (g - g_eq(p*, u)))_k with Omega = M^-1 S M:
 * the bracket of eq. viscousForce, before the factor -nu/cs^2 and the
 * contraction with grad(rho).                                          */
static void viscous_bracket(orc_lat L, const double *g, double s_nu, const double u[3], double V[3][3])
{
    const orc_mrt *m = build_mrt_q(L.q);
    double pstar = 0.0;
    for (int i = 0; i < L.q; ++i) pstar += g[i];
    double geq[QMAX], d[QMAX], mm[QMAX], Sd[QMAX], om[QMAX], S[QMAX];
    hydro_equilibrium(L, pstar, u, geq);
    for (int i = 0; i < L.q; ++i) d[i] = g[i] - geq[i];
    relaxation_rates(m, s_nu, S);
    matvec(m, m->M, d, mm);
    for (int k = 0; k < L.q; ++k) Sd[k] = S[k] * mm[k];
    matvec(m, m->Minv, Sd, om);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int i = 0; i < L.q; ++i) s += L.e[i][a] * L.e[i][b] * om[i];
            V[a][b] = s;
        }
}

int orc_viscous_bracket(const double *g, double s_nu, const double *u, double *V)
{
    if (build_mrt() != 0) return -1;
    double v[3][3];
    viscous_bracket(lat_of(Q27), g, s_nu, u, v);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) V[3 * a + b] = v[a][b];
    return 0;
}

/* Moment-space collision (eq. improved_collision, with the "m -" of the
 * listing): m = M g, m_eq = M g_eq(p*, u), F_m = (0, F/rho, 0, ...),
 * m* = m - S (m - m_eq + F_m/2) + F_m, g* = M^-1 m*.                  */
static void mrt_collide(orc_lat L, const double *g, double pstar, const double u[3],
                        const double F[3], double rho, double s_nu, double *out)
{
    const orc_mrt *m = build_mrt_q(L.q);
    double geq[QMAX], mm[QMAX], meq[QMAX], Fm[QMAX], ms[QMAX], S[QMAX];
    hydro_equilibrium(L, pstar, u, geq);
    matvec(m, m->M, g, mm);
    matvec(m, m->M, geq, meq);
    relaxation_rates(m, s_nu, S);
    /* F_m is F/rho on the three first-order rows (the monomials x, y, z,
     * already orthogonal to row 0) and zero on every other row.        */
    for (int k = 0; k < L.q; ++k) {
        Fm[k] = 0.0;
        if (m->deg[k] == 1)
            for (int a = 0; a < 3; ++a)
                if (m->expo[k][a] == 1) Fm[k] = F[a] / rho;
    }
    for (int k = 0; k < L.q; ++k) ms[k] = mm[k] - S[k] * (mm[k] - meq[k] + 0.5 * Fm[k]) + Fm[k];
    matvec(m, m->Minv, ms, out);
}

int orc_mrt_collide(const double *g, double pstar, const double *u, const double *F,
                    double rho, double s_nu, double *out)
{
    if (build_mrt() != 0) return -1;
    mrt_collide(lat_of(Q27), g, pstar, u, F, rho, s_nu, out);
    return 0;
}

/* Hydrodynamic equilibrium, collision and viscous bracket on a velocity set
 * of q directions (pins of the other lattices).                            */
int orc_hydro_equilibrium_q(int32_t q, double pstar, const double *u, double *out)
{
    if (q != Q15 && q != Q19 && q != Q27) return -1;
    init_weights();
    hydro_equilibrium(lat_of(q), pstar, u, out);
    return 0;
}

int orc_mrt_collide_q(int32_t q, const double *g, double pstar, const double *u, const double *F, double rho,
                      double s_nu, double *out)
{
    if ((q != Q15 && q != Q19 && q != Q27) || !build_mrt_q(q)) return -1;
    mrt_collide(lat_of(q), g, pstar, u, F, rho, s_nu, out);
    return 0;
}

int orc_viscous_bracket_q(int32_t q, const double *g, double s_nu, const double *u, double *V)
{
    if ((q != Q15 && q != Q19 && q != Q27) || !build_mrt_q(q)) return -1;
    double v[3][3];
    viscous_bracket(lat_of(q), g, s_nu, u, v);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) V[3 * a + b] = v[a][b];
    return 0;
}

/* Phase-field collision (eq. lb_interface), h* = h + Omega (h_eq - h - F/2)
 * + F with Omega = R^-1 S R in raw moments: the first-order moments relax
 * with omega, every other moment with one (Sec. 3.1).  The collision of
 * the fused and straightforward steps with phase_mrt = 1.                  */
static void phase_mrt_collide(orc_lat L, const double *h, const double *heq, const double *F, double omega,
                              double *out)
{
    const orc_mrt *m = build_mrt_q(L.q);
    double d[QMAX], md[QMAX];
    for (int i = 0; i < L.q; ++i) d[i] = heq[i] - h[i] - 0.5 * F[i];
    matvec(m, m->R, d, md);
    for (int k = 0; k < L.q; ++k) md[k] *= (m->deg[k] == 1) ? omega : 1.0;
    matvec(m, m->Rinv, md, out);
    for (int i = 0; i < L.q; ++i) out[i] += h[i] + F[i];
}

int orc_phase_mrt_collide_q(int32_t q, const double *h, const double *heq, const double *F, double omega,
                            double *out)
{
    if ((q != Q15 && q != Q19 && q != Q27) || !build_mrt_q(q)) return -1;
    phase_mrt_collide(lat_of(q), h, heq, F, omega, out);
    return 0;
}

/* ---- grid --------------------------------------------------------------- */
typedef struct {
    orc_params p;
    int64_t n;
    double *H, *Hn;      /* 15 planes: post-collision phase PDFs at x */
    double *G, *Gn;      /* 27 planes: pre-collision hydro PDFs at x */
    double *phiA, *phiB; /* phase field, previous / new               */
    double *u;           /* 3 planes                                   */
    int qp, qh;          /* velocity sets of the two steps              */
} orc_state;

static inline int64_t cidx(const orc_params *p, int x, int y, int z)
{
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * z);
}

static inline int wrap(int v, int n) { return ((v % n) + n) % n; }

static inline int is_wall_row(const orc_params *p, int y)
{
    return p->walls_y && (y == 0 || y == p->ny - 1);
}

/* Neighbour y coordinate: periodic without walls; with walls rows 0 and
 * ny-1 exist as solid rows and fluid rows never step past them.        */
static inline int ny_nb(const orc_params *p, int y, int dy)
{
    return p->walls_y ? y + dy : wrap(y + dy, p->ny);
}

/* phi at x + d for the finite-difference stencils; a wall row is replaced
 * by its mirror image about the wall, which is the current fluid row.  */
static inline double phi_at(const orc_params *p, const double *phi, int x, int y, int z,
                            int dx, int dy, int dz)
{
    int yy = ny_nb(p, y, dy);
    if (is_wall_row(p, yy)) yy = y;
    return phi[cidx(p, wrap(x + dx, p->nx), yy, wrap(z + dz, p->nz))];
}

/* Isotropic gradient (eq. grad): (1/cs^2) sum_i w_i e_i phi(x + e_i),
 * evaluated as sum over the half set of w_i e_i (phi(x+e_i) - phi(x-e_i)). */
static void iso_gradient(const orc_params *p, const double *phi, int q, int x, int y, int z,
                         double grad[3])
{
    const orc_lat L = lat_of(q);
    const int (*E)[3] = L.e;
    const double *W = L.w;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = 1; i < q; i += 2) {
        double d = phi_at(p, phi, x, y, z, E[i][0], E[i][1], E[i][2]) -
                   phi_at(p, phi, x, y, z, -E[i][0], -E[i][1], -E[i][2]);
        for (int a = 0; a < 3; ++a) acc[a] += W[i] * E[i][a] * d;
    }
    for (int a = 0; a < 3; ++a) grad[a] = acc[a] / CS2;
}

/* Isotropic Laplacian (eq. lap): (2/cs^2) sum_i w_i [phi(x+e_i) - phi(x)]. */
/* Density and relaxation time of a cell (eq. density and the tau
 * interpolation of Sec. 3.2): linear in phi between the two bulk phases.
 * The interpolation is defined on [phi_L, phi_H]; the conservative
 * Allen-Cahn model overshoots that interval by ~1e-3 (most in the cores of
 * small bubbles, where |grad phi| ~ 0), and at rho_H/rho_L = 1000 an
 * undershoot of 1e-3 would put rho near zero.  phi is therefore clamped to
 * the interval before interpolating, which keeps rho in [rho_L, rho_H],
 * unless density_literal asks for the formula as printed.                 */
static double phase_clamp(const orc_params *p, double phi)
{
    if (p->density_literal) return phi;
    const double lo = p->phi_L < p->phi_H ? p->phi_L : p->phi_H;
    const double hi = p->phi_L < p->phi_H ? p->phi_H : p->phi_L;
    return phi < lo ? lo : (phi > hi ? hi : phi);
}

static double density_of(const orc_params *p, double phi)
{
    return p->rho_L + (phase_clamp(p, phi) - p->phi_L) * (p->rho_H - p->rho_L) / (p->phi_H - p->phi_L);
}

static double iso_laplacian(const orc_params *p, const double *phi, int q, int x, int y, int z)
{
    const orc_lat L = lat_of(q);
    const int (*E)[3] = L.e;
    const double *W = L.w;
    double c = phi[cidx(p, x, y, z)];
    double acc = 0.0;
    for (int i = 0; i < q; ++i)
        acc += W[i] * (phi_at(p, phi, x, y, z, E[i][0], E[i][1], E[i][2]) - c);
    return 2.0 * acc / CS2;
}

/* Stencil queries on a caller field, for the finite-difference pins. */
void orc_stencil(const orc_params *p, const double *phi, int32_t q, int32_t x, int32_t y,
                 int32_t z, double *grad, double *lap)
{
    init_weights();
    iso_gradient(p, phi, q, x, y, z, grad);
    *lap = iso_laplacian(p, phi, q, x, y, z);
}

/* ---- state lifecycle ------------------------------------------------------ */
orc_state *orc_create(const orc_params *p)
{
    if (!p || p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return NULL;
    if (p->walls_y && p->ny < 3) return NULL;
    const int qp = p->lattice_phase == 0 ? Q15 : p->lattice_phase;
    const int qh = p->lattice_hydro == 0 ? Q27 : p->lattice_hydro;
    if ((qp != Q15 && qp != Q19 && qp != Q27) || (qh != Q15 && qh != Q19 && qh != Q27)) return NULL;
    if (build_mrt() != 0 || !build_mrt_q(qp) || !build_mrt_q(qh)) return NULL;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->p = *p;
    s->qp = qp;
    s->qh = qh;
    s->n = (int64_t)p->nx * p->ny * p->nz;
    size_t n = (size_t)s->n;
    s->H = calloc((size_t)qp * n, sizeof(double));
    s->Hn = calloc((size_t)qp * n, sizeof(double));
    s->G = calloc((size_t)qh * n, sizeof(double));
    s->Gn = calloc((size_t)qh * n, sizeof(double));
    s->phiA = calloc(n, sizeof(double));
    s->phiB = calloc(n, sizeof(double));
    s->u = calloc(3 * n, sizeof(double));
    if (!s->H || !s->Hn || !s->G || !s->Gn || !s->phiA || !s->phiB || !s->u) {
        free(s->H); free(s->Hn); free(s->G); free(s->Gn);
        free(s->phiA); free(s->phiB); free(s->u); free(s);
        return NULL;
    }
    return s;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    free(s->H); free(s->Hn); free(s->G); free(s->Gn);
    free(s->phiA); free(s->phiB); free(s->u); free(s);
}

/* Initial state: h = phi Gamma(u) taken as post-collision, g = g_eq(p*, u)
 * taken as pre-collision, phi_A = phi, u = u.  Wall cells hold zeros.   */
void orc_init(orc_state *s, const double *phi, const double *u, const double *pstar)
{
    const orc_params *p = &s->p;
    int64_t n = s->n;
    const orc_lat LP = lat_of(s->qp), LH = lat_of(s->qh);
    memset(s->H, 0, sizeof(double) * LP.q * n);
    memset(s->G, 0, sizeof(double) * LH.q * n);
    memset(s->Hn, 0, sizeof(double) * LP.q * n);
    memset(s->Gn, 0, sizeof(double) * LH.q * n);
    memset(s->phiA, 0, sizeof(double) * n);
    memset(s->phiB, 0, sizeof(double) * n);
    memset(s->u, 0, sizeof(double) * 3 * n);
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                if (is_wall_row(p, y)) continue;
                int64_t c = cidx(p, x, y, z);
                double uc[3] = {u[c], u[n + c], u[2 * n + c]};
                double geq[QMAX];
                for (int i = 0; i < LP.q; ++i) s->H[i * n + c] = phi[c] * gamma_i(LP.e[i], LP.w[i], uc);
                hydro_equilibrium(LH, pstar[c], uc, geq);
                for (int i = 0; i < LH.q; ++i) s->G[i * n + c] = geq[i];
                s->phiA[c] = phi[c];
                for (int a = 0; a < 3; ++a) s->u[a * n + c] = uc[a];
            }
}

/* ---- phase-field step (pull, sum, collide) ------------------------------ */
static void phase_cell(orc_state *s, int x, int y, int z)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n;
    const int64_t c = cidx(p, x, y, z);
    const orc_lat L = lat_of(s->qp);
    double P[QMAX];
    for (int i = 0; i < L.q; ++i) {
        int sy = ny_nb(p, y, -L.e[i][1]);
        if (is_wall_row(p, sy)) {
            P[i] = s->H[opposite(i) * n + c]; /* halfway bounce-back */
        } else {
            int64_t src = cidx(p, wrap(x - L.e[i][0], p->nx), sy, wrap(z - L.e[i][2], p->nz));
            P[i] = s->H[i * n + src];
        }
    }
    double phi = 0.0;
    for (int i = 0; i < L.q; ++i) phi += P[i];
    s->phiB[c] = phi;

    double grad[3];
    iso_gradient(p, s->phiA, L.q, x, y, z, grad);
    double gnorm = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    double nrm[3];
    for (int a = 0; a < 3; ++a) nrm[a] = grad[a] / (gnorm + p->normal_eps);
    double phi0 = 0.5 * (p->phi_L + p->phi_H);
    double dphi = s->phiA[c] - phi0;
    double theta = (1.0 - 4.0 * dphi * dphi) / p->xi;

    double uc[3] = {s->u[c], s->u[n + c], s->u[2 * n + c]};
    double tau_phi = p->mobility / CS2;            /* eq. mobility, dt = 1 */
    double omega = 1.0 / (tau_phi + 0.5);
    double Fphi[QMAX];
    phase_forcing(L, theta, nrm, Fphi);
    if (p->phase_mrt) {
        double heq[QMAX], hs[QMAX];
        for (int i = 0; i < L.q; ++i) heq[i] = phi * gamma_i(L.e[i], L.w[i], uc);
        phase_mrt_collide(L, P, heq, Fphi, omega, hs);
        for (int i = 0; i < L.q; ++i) s->Hn[i * n + c] = hs[i];
    } else {
        for (int i = 0; i < L.q; ++i) {
            double heq = phi * gamma_i(L.e[i], L.w[i], uc);
            s->Hn[i * n + c] = P[i] + omega * (heq - P[i] - 0.5 * Fphi[i]) + Fphi[i];
        }
    }
}

/* ---- hydrodynamic step (collide, push, velocity update) ----------------- */
static void hydro_cell(orc_state *s, int x, int y, int z)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n;
    const int64_t c = cidx(p, x, y, z);
    const orc_lat L = lat_of(s->qh);
    double g[QMAX];
    for (int i = 0; i < L.q; ++i) g[i] = s->G[i * n + c];

    const double dphi = p->phi_H - p->phi_L;
    double phi = s->phiB[c];
    double rho = density_of(p, phi);
    double tau = p->tau_L + (phase_clamp(p, phi) - p->phi_L) * (p->tau_H - p->tau_L) / dphi;
    double s_nu = 1.0 / (tau + 0.5);
    double nu = tau * CS2;

    double grad[3];
    iso_gradient(p, s->phiB, L.q, x, y, z, grad);
    double lap = iso_laplacian(p, s->phiB, L.q, x, y, z);
    double grad_rho[3];
    for (int a = 0; a < 3; ++a) grad_rho[a] = (p->rho_H - p->rho_L) / dphi * grad[a];

    double beta = 12.0 * p->sigma / p->xi;
    double kappa = 1.5 * p->sigma * p->xi;
    double phi0 = 0.5 * (p->phi_L + p->phi_H);
    double mu_phi = 4.0 * beta * (phi - p->phi_L) * (phi - p->phi_H) * (phi - phi0) - kappa * lap;

    double pstar = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L.q; ++i) {
        pstar += g[i];
        for (int a = 0; a < 3; ++a) j[a] += g[i] * L.e[i][a];
    }

    double u_old[3] = {s->u[c], s->u[n + c], s->u[2 * n + c]};
    double V[3][3];
    viscous_bracket(L, g, s_nu, u_old, V);

    double F[3];
    for (int a = 0; a < 3; ++a) {
        double Fp = -pstar * CS2 * grad_rho[a];
        double Fs = mu_phi * grad[a];
        double Fmu = 0.0;
        for (int b = 0; b < 3; ++b) Fmu += V[a][b] * grad_rho[b];
        Fmu *= -nu / CS2;
        double Fb = (rho - p->rho_ref) * p->accel[a];
        F[a] = Fp + Fs + Fmu + Fb;
    }

    double u_new[3];
    for (int a = 0; a < 3; ++a) u_new[a] = j[a] + F[a] / (2.0 * rho);
    for (int a = 0; a < 3; ++a) s->u[a * n + c] = u_new[a];

    double gs[QMAX];
    mrt_collide(L, g, pstar, u_new, F, rho, s_nu, gs);

    for (int i = 0; i < L.q; ++i) {
        int dy = ny_nb(p, y, L.e[i][1]);
        if (is_wall_row(p, dy)) {
            s->Gn[opposite(i) * n + c] = gs[i]; /* halfway bounce-back */
        } else {
            int64_t dst = cidx(p, wrap(x + L.e[i][0], p->nx), dy, wrap(z + L.e[i][2], p->nz));
            s->Gn[i * n + dst] = gs[i];
        }
    }
}

static void swap_ptr(double **a, double **b) { double *t = *a; *a = *b; *b = t; }

/* One coupled time step: phase pass over all fluid cells, then hydro pass,
 * then the buffer swap.  Cells are independent within a pass, so the
 * result does not depend on the number of threads.                     */
void orc_step(orc_state *s, int32_t nsteps)
{
    const orc_params *p = &s->p;
    const int nyz = p->ny * p->nz;
    for (int t = 0; t < nsteps; ++t) {
#pragma omp parallel for schedule(static)
        for (int yz = 0; yz < nyz; ++yz) {
            int y = yz % p->ny, z = yz / p->ny;
            if (is_wall_row(p, y)) continue;
            for (int x = 0; x < p->nx; ++x) phase_cell(s, x, y, z);
        }
#pragma omp parallel for schedule(static)
        for (int yz = 0; yz < nyz; ++yz) {
            int y = yz % p->ny, z = yz / p->ny;
            if (is_wall_row(p, y)) continue;
            for (int x = 0; x < p->nx; ++x) hydro_cell(s, x, y, z);
        }
        swap_ptr(&s->H, &s->Hn);
        swap_ptr(&s->G, &s->Gn);
        swap_ptr(&s->phiA, &s->phiB);
    }
}

/* ---- straightforward algorithm (Alg. naiveAlgorithm, Sec. 4.2) ---------
 * The six steps of the straightforward algorithm, each a pass of its own
 * over all fluid cells: collide h, collide g, stream h, update phi, stream
 * g, update u.  Read as a time-consistent scheme: every collision of step t
 * takes phi, grad(phi), theta and u of time t, and the velocity update
 * takes the streamed g and the new phi, with the stored velocity (of the
 * previous time) inside the viscous force, as in the fused step.  The
 * collision of g recomputes the force from the state it collides (its
 * moments, phi and the updated u).
 *
 * The loop is cut where the canonical state of the fused step sits (h
 * post-collision at the cell, g pre-collision and already streamed), so one
 * call runs: stream h, update phi, update u, collide h, collide g and
 * stream g (push).  The initial state is the same as the fused step's.    */

/* Force of eq. forceHydro at cell c from the pre-collision g there, the
 * phase field `phi` (stencil) and the velocity `uv` inside the viscous
 * force; also returns rho, s_nu and the moments p* and j.                 */
static void naive_force(const orc_state *s, const double *phi, int x, int y, int z, const double *g,
                        const double uv[3], double F[3], double *rho_out, double *s_nu_out,
                        double *pstar_out, double j[3])
{
    const orc_params *p = &s->p;
    const int64_t c = cidx(p, x, y, z);
    const double dphi = p->phi_H - p->phi_L;
    double ph = phi[c];
    double rho = density_of(p, ph);
    double tau = p->tau_L + (phase_clamp(p, ph) - p->phi_L) * (p->tau_H - p->tau_L) / dphi;
    double s_nu = 1.0 / (tau + 0.5);
    double nu = tau * CS2;

    double grad[3];
    const orc_lat L = lat_of(s->qh);
    iso_gradient(p, phi, L.q, x, y, z, grad);
    double lap = iso_laplacian(p, phi, L.q, x, y, z);
    double grad_rho[3];
    for (int a = 0; a < 3; ++a) grad_rho[a] = (p->rho_H - p->rho_L) / dphi * grad[a];
    double beta = 12.0 * p->sigma / p->xi;
    double kappa = 1.5 * p->sigma * p->xi;
    double phi0 = 0.5 * (p->phi_L + p->phi_H);
    double mu_phi = 4.0 * beta * (ph - p->phi_L) * (ph - p->phi_H) * (ph - phi0) - kappa * lap;

    double pstar = 0.0;
    for (int a = 0; a < 3; ++a) j[a] = 0.0;
    for (int i = 0; i < L.q; ++i) {
        pstar += g[i];
        for (int a = 0; a < 3; ++a) j[a] += g[i] * L.e[i][a];
    }
    double V[3][3];
    viscous_bracket(L, g, s_nu, uv, V);
    for (int a = 0; a < 3; ++a) {
        double Fp = -pstar * CS2 * grad_rho[a];
        double Fs = mu_phi * grad[a];
        double Fmu = 0.0;
        for (int b = 0; b < 3; ++b) Fmu += V[a][b] * grad_rho[b];
        Fmu *= -nu / CS2;
        double Fb = (rho - p->rho_ref) * p->accel[a];
        F[a] = Fp + Fs + Fmu + Fb;
    }
    *rho_out = rho;
    *s_nu_out = s_nu;
    *pstar_out = pstar;
}

/* Stream h: the pre-collision population of direction i at x is the
 * post-collision one of x - e_i (halfway bounce-back at a wall).         */
static void naive_stream_h(orc_state *s, int x, int y, int z)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n, c = cidx(p, x, y, z);
    const orc_lat L = lat_of(s->qp);
    for (int i = 0; i < L.q; ++i) {
        int sy = ny_nb(p, y, -L.e[i][1]);
        if (is_wall_row(p, sy))
            s->Hn[i * n + c] = s->H[opposite(i) * n + c];
        else
            s->Hn[i * n + c] = s->H[i * n + cidx(p, wrap(x - L.e[i][0], p->nx), sy, wrap(z - L.e[i][2], p->nz))];
    }
}

/* Update phi = sum of the streamed populations (eq. updatePhaseField). */
static void naive_update_phi(orc_state *s, int x, int y, int z)
{
    const int64_t n = s->n, c = cidx(&s->p, x, y, z);
    double phi = 0.0;
    for (int i = 0; i < s->qp; ++i) phi += s->Hn[i * n + c];
    s->phiB[c] = phi;
}

/* Update u = j + F/(2 rho) (eq. updateVelocityField) from the streamed g
 * and the new phi; the stored velocity enters the viscous force.         */
static void naive_update_u(orc_state *s, int x, int y, int z)
{
    const int64_t n = s->n, c = cidx(&s->p, x, y, z);
    double g[QMAX];
    for (int i = 0; i < s->qh; ++i) g[i] = s->G[i * n + c];
    double u_old[3] = {s->u[c], s->u[n + c], s->u[2 * n + c]};
    double F[3], rho, s_nu, pstar, j[3];
    naive_force(s, s->phiB, x, y, z, g, u_old, F, &rho, &s_nu, &pstar, j);
    for (int a = 0; a < 3; ++a) s->u[a * n + c] = j[a] + F[a] / (2.0 * rho);
}

/* Collide h (eq. lb_interface with F^phi of eq. interfaceTracking): phi,
 * grad(phi), theta and u all of the new time.                            */
static void naive_collide_h(orc_state *s, int x, int y, int z)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n, c = cidx(p, x, y, z);
    double phi = s->phiB[c];
    double grad[3];
    const orc_lat L = lat_of(s->qp);
    iso_gradient(p, s->phiB, L.q, x, y, z, grad);
    double gnorm = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    double nrm[3];
    for (int a = 0; a < 3; ++a) nrm[a] = grad[a] / (gnorm + p->normal_eps);
    double phi0 = 0.5 * (p->phi_L + p->phi_H);
    double theta = (1.0 - 4.0 * (phi - phi0) * (phi - phi0)) / p->xi;
    double uc[3] = {s->u[c], s->u[n + c], s->u[2 * n + c]};
    double omega = 1.0 / (p->mobility / CS2 + 0.5);
    double Fphi[QMAX];
    phase_forcing(L, theta, nrm, Fphi);
    if (p->phase_mrt) {
        double hh[QMAX], heq[QMAX], hs[QMAX];
        for (int i = 0; i < L.q; ++i) {
            hh[i] = s->Hn[i * n + c];
            heq[i] = phi * gamma_i(L.e[i], L.w[i], uc);
        }
        phase_mrt_collide(L, hh, heq, Fphi, omega, hs);
        for (int i = 0; i < L.q; ++i) s->H[i * n + c] = hs[i];
    } else {
        for (int i = 0; i < L.q; ++i) {
            double h = s->Hn[i * n + c];
            double heq = phi * gamma_i(L.e[i], L.w[i], uc);
            s->H[i * n + c] = h + omega * (heq - h - 0.5 * Fphi[i]) + Fphi[i];
        }
    }
}

/* Collide g (eq. improved_collision) with the force recomputed from the
 * state it collides, then push it to x + e_i (bounce-back at a wall).     */
static void naive_collide_g(orc_state *s, int x, int y, int z)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n, c = cidx(p, x, y, z);
    double g[QMAX];
    for (int i = 0; i < s->qh; ++i) g[i] = s->G[i * n + c];
    double uc[3] = {s->u[c], s->u[n + c], s->u[2 * n + c]};
    double F[3], rho, s_nu, pstar, j[3];
    naive_force(s, s->phiB, x, y, z, g, uc, F, &rho, &s_nu, &pstar, j);
    const orc_lat L = lat_of(s->qh);
    double gs[QMAX];
    mrt_collide(L, g, pstar, uc, F, rho, s_nu, gs);
    for (int i = 0; i < L.q; ++i) {
        int dy = ny_nb(p, y, L.e[i][1]);
        if (is_wall_row(p, dy))
            s->Gn[opposite(i) * n + c] = gs[i];
        else
            s->Gn[i * n + cidx(p, wrap(x + L.e[i][0], p->nx), dy, wrap(z + L.e[i][2], p->nz))] = gs[i];
    }
}

#define ORC_FLUID_PASS(fn)                                                   \
    _Pragma("omp parallel for schedule(static)")                             \
    for (int yz = 0; yz < p->ny * p->nz; ++yz) {                             \
        int y = yz % p->ny, z = yz / p->ny;                                  \
        if (is_wall_row(p, y)) continue;                                     \
        for (int x = 0; x < p->nx; ++x) fn(s, x, y, z);                      \
    }

void orc_step_naive(orc_state *s, int32_t nsteps)
{
    const orc_params *p = &s->p;
    for (int t = 0; t < nsteps; ++t) {
        ORC_FLUID_PASS(naive_stream_h)
        ORC_FLUID_PASS(naive_update_phi)
        ORC_FLUID_PASS(naive_update_u)
        ORC_FLUID_PASS(naive_collide_h)
        ORC_FLUID_PASS(naive_collide_g)
        swap_ptr(&s->G, &s->Gn);
        swap_ptr(&s->phiA, &s->phiB);
    }
}
#undef ORC_FLUID_PASS

/* Canonical state: H (post-collision phase PDFs), G (pre-collision hydro
 * PDFs), phi_A (latest phase field), u (latest velocity). Any pointer may
 * be NULL.                                                             */
void orc_get_state(const orc_state *s, double *H, double *G, double *phi, double *u)
{
    size_t n = (size_t)s->n;
    if (H) memcpy(H, s->H, sizeof(double) * s->qp * n);
    if (G) memcpy(G, s->G, sizeof(double) * s->qh * n);
    if (phi) memcpy(phi, s->phiA, sizeof(double) * n);
    if (u) memcpy(u, s->u, sizeof(double) * 3 * n);
}

void orc_set_state(orc_state *s, const double *H, const double *G, const double *phi,
                   const double *u)
{
    size_t n = (size_t)s->n;
    if (H) memcpy(s->H, H, sizeof(double) * s->qp * n);
    if (G) memcpy(s->G, G, sizeof(double) * s->qh * n);
    if (phi) memcpy(s->phiA, phi, sizeof(double) * n);
    if (u) memcpy(s->u, u, sizeof(double) * 3 * n);
}

/* Moves the state to new macroscopic fields phi', u' and pressure p'
 * keeping each population's non-equilibrium part (its distance from the
 * equilibria of Section 3): in every fluid cell
 *   H_i += phi' Gamma_i(u') - phi Gamma_i(u),
 *   G_i += g^eq_i(p*', u') - g^eq_i(p*, u),
 * with phi, u the current phase field and velocity, p* = sum_i G_i and
 * p*' = p' / (rho(phi') cs^2); then phi_A = phi', u = u'.  Wall cells are
 * unchanged.                                                            */
void orc_shift_equilibrium(orc_state *s, const double *phi, const double *u, const double *pres)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n;
    const orc_lat LP = lat_of(s->qp), LH = lat_of(s->qh);
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                if (is_wall_row(p, y)) continue;
                const int64_t c = cidx(p, x, y, z);
                const double u0[3] = {s->u[c], s->u[n + c], s->u[2 * n + c]};
                const double u1[3] = {u[c], u[n + c], u[2 * n + c]};
                const double phi0 = s->phiA[c], phi1 = phi[c];
                for (int i = 0; i < LP.q; ++i)
                    s->H[i * n + c] += phi1 * gamma_i(LP.e[i], LP.w[i], u1) - phi0 * gamma_i(LP.e[i], LP.w[i], u0);
                double ps0 = 0.0;
                for (int i = 0; i < LH.q; ++i) ps0 += s->G[i * n + c];
                const double ps1 = pres[c] / (density_of(p, phi1) * CS2);
                double e0[QMAX], e1[QMAX];
                hydro_equilibrium(LH, ps0, u0, e0);
                hydro_equilibrium(LH, ps1, u1, e1);
                for (int i = 0; i < LH.q; ++i) s->G[i * n + c] += e1[i] - e0[i];
                s->phiA[c] = phi1;
                for (int a = 0; a < 3; ++a) s->u[a * n + c] = u1[a];
            }
}

/* Equilibrium state of given macroscopic fields with the pressure p
 * instead of p*: the initial-state rule of orc_init with
 * p* = p / (rho(phi) cs^2) (Section 3.2), rho from eq. density as in the
 * step.  Wall cells hold zeros.                                          */
void orc_init_pressure(orc_state *s, const double *phi, const double *u, const double *pres)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n;
    double *ps = (double *)calloc((size_t)n, sizeof(double));
    if (!ps) return;
    for (int64_t c = 0; c < n; ++c) {
        int y = (int)((c / p->nx) % p->ny);
        if (is_wall_row(p, y)) continue;
        ps[c] = pres[c] / (density_of(p, phi[c]) * CS2);
    }
    orc_init(s, phi, u, ps);
    free(ps);
}

/* Pressure p = p* rho cs^2 with p* = sum_i g_i (Section 3.2). */
void orc_pressure(const orc_state *s, double *pout)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n;
    for (int64_t c = 0; c < n; ++c) {
        int y = (int)((c / p->nx) % p->ny);
        if (is_wall_row(p, y)) { pout[c] = 0.0; continue; }
        double ps = 0.0;
        for (int i = 0; i < s->qh; ++i) ps += s->G[i * n + c];
        double rho = density_of(p, s->phiA[c]);
        pout[c] = ps * rho * CS2;
    }
}

/* Diagnostics over fluid cells, FP64, serial in z, y, x order.
 * chi = (phi_H - phi)/(phi_H - phi_L) marks the light phase; the centroid
 * and rise velocity are chi-weighted means; xi_eff = sum 4chi(1-chi) /
 * sum |grad phi|/(phi_H - phi_L), which equals xi for the planar
 * equilibrium profile; the gradient is the D3Q27 isotropic one.       */
void orc_stats_compute(const orc_state *s, orc_stats *out)
{
    const orc_params *p = &s->p;
    const int64_t n = s->n;
    const double dphi = p->phi_H - p->phi_L;
    memset(out, 0, sizeof(*out));
    double cx = 0.0, cy = 0.0, cz = 0.0, ury = 0.0;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y) {
            if (is_wall_row(p, y)) continue;
            for (int x = 0; x < p->nx; ++x) {
                int64_t c = cidx(p, x, y, z);
                double phi = s->phiA[c];
                double rho = density_of(p, phi);
                double ux = s->u[c], uy = s->u[n + c], uz = s->u[2 * n + c];
                double chi = (p->phi_H - phi) / dphi;
                double grad[3];
                iso_gradient(p, s->phiA, Q27, x, y, z, grad);
                double gn = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
                double sp = sqrt(ux * ux + uy * uy + uz * uz);
                out->mass += phi;
                out->momentum[0] += rho * ux;
                out->momentum[1] += rho * uy;
                out->momentum[2] += rho * uz;
                out->gas_volume += chi;
                cx += chi * x;
                cy += chi * y;
                cz += chi * z;
                ury += chi * uy;
                out->interface_sum += 4.0 * chi * (1.0 - chi);
                out->grad_sum += gn / dphi;
                if (sp > out->max_speed) out->max_speed = sp;
            }
        }
    if (out->gas_volume != 0.0) {
        out->centroid[0] = cx / out->gas_volume;
        out->centroid[1] = cy / out->gas_volume;
        out->centroid[2] = cz / out->gas_volume;
        out->rise_velocity = ury / out->gas_volume;
    }
    out->xi_eff = (out->grad_sum != 0.0) ? out->interface_sum / out->grad_sum : 0.0;
}

int64_t orc_num_cells(const orc_state *s) { return s->n; }

/* Threads the OpenMP cell loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
