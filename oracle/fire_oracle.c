/*
 * fire_oracle.c -- plain FP64 CPU oracle of the WRF-Fire fire-mesh time step
 * (Mandel, Beezley & Kochanski, "Coupled atmosphere-wildland fire modeling
 * with WRF-Fire version 3.3", arXiv:1102.1343).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the product
 * library never links it, and the two share no source, header or table.
 *
 * Every step is written as plain loops over the fire mesh, in double
 * precision, in the order Sect. 6 gives for one time step of the fire model:
 * (1) ignition, (2) Heun step of the level-set equation, (3) ignition times,
 * (4) fuel fraction, (5) heat fluxes, (6) averaging onto the atmosphere mesh,
 * plus the boundary check of Sect. 4.1.  OpenMP only splits independent
 * per-cell loops, so results do not depend on the thread count.
 *
 * Where the paper is silent or garbled the reading used is stated at the
 * point of use and tagged R1..R28, one tag per reading, so the same choice can
 * be found in the HIP path.
 *
 * Parity status per function (what pins it, see tests/test_oracle_*.py):
 *   ghost / oracle_extrapolate     pinned: hand-built ghost fixtures
 *   oracle_godunov                 pinned: branch table of Eq. (13), monotone-
 *                                  scheme identity max(D-^+,D+^-)
 *   oracle_ros (coefficient form)  pinned: chaparral values of Eq. (2);
 *                                  equality with the product form Eq. (1)
 *   rothermel_chain / oracle_coef  pinned: every intermediate of Table 2
 *   (Rothermel chain, Table 2)     (sigma ... R0, C, B, E, phi_W, phi_S, S)
 *                                  against a hand evaluation of the printed
 *                                  formulas for two fuels
 *                                  (tests/golden/rothermel_table2.txt), limit
 *                                  cases of readings R1/R2, extinction
 *                                  moisture (R0 = 0), linearity in h
 *   level set (Heun/Godunov/ROS)   pinned: planar-front closed form, circle
 *                                  r0 + S t convergence, Heun time order
 *   ignition time Eq. (14)         pinned: planar-front closed form
 *   ignition Eqs. (20)-(21)        pinned: brute-force segment distance
 *   fuel fraction Eqs. (15)-(19)   pinned: F = 1 off fire, exponential decay
 *                                  Eq. (4), exact beta cases, O(h^2) test
 *   fluxes/averaging Eqs. (5)-(6)  pinned: exact telescoping conservation
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- data passed in from the Python wrapper (layouts mirrored there) ---- */

typedef struct {              /* one fuel category, Table 1 quantities, SI units */
    double windrf;            /* a: wind reduction 6.1 m -> midflame          */
    double tf;                /* T_f (s); if <= 0 it is derived from weight    */
    double weight;            /* w (s)                                         */
    double fgi;               /* w_l total fuel load (kg/m^2)                  */
    double fueldepthm;        /* delta (m)                                     */
    double savr;              /* sigma (1/m)                                   */
    double fuelmce;           /* M_x                                           */
    double fueldens;          /* rho_P (kg/m^3)                                */
    double st;                /* S_T                                           */
    double se;                /* S_E                                           */
    double cmbcnst;           /* h (J/kg)                                      */
    double fuelmc_g;          /* M_f                                           */
    double ros_mult;          /* per-category spread multiplier m_k            */
    int32_t ichap;            /* 1: chaparral rate, Eq. (2)                    */
    int32_t pad_;
} of_fuel;

typedef struct {              /* segment / drip-torch ignition, Sect. 4.4     */
    double ax, ay, bx, by;    /* segment end points (m); b unused for a torch */
    double t_start;           /* t_g (s)                                      */
    double radius;            /* r_g (m)                                      */
    double ros;               /* S_g (m/s); +inf = instantaneous              */
    double vx, vy;            /* drip-torch velocity (m/s); 0,0 = segment     */
    double t_end;             /* t_h (s), drip torch only                     */
} of_ign;

typedef struct {
    int32_t nx, ny;           /* fire mesh cells                              */
    double dx, dy;            /* fire mesh spacing (m)                        */
    int32_t sr_x, sr_y;       /* fire cells per atmosphere cell               */
} of_mesh;

typedef struct {
    double viscosity;         /* epsilon of Eq. (12)                          */
    int32_t viscosity_mode;   /* 0: eps*S*Lap (reading R9), 1: eps*Lap        */
    int32_t guard_width;      /* boundary guard ring width (cells)            */
    double ros_cap;           /* upper cap on S (reading R23), may be +inf    */
} of_prm;

/* coefficient table row layout, one row of OC_N doubles per category */
enum { OC_S0, OC_R0, OC_B, OC_C, OC_D, OC_E, OC_M, OC_TF, OC_CH, OC_CQ, OC_N };

enum { OS_BOUNDARY = 1, OS_NONFINITE = 2 };

int oracle_ncoef(void) { return OC_N; }
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the oracle's parallel loops from now on (n >= 1). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
int oracle_sizeof_fuel(void) { return (int)sizeof(of_fuel); }
int oracle_sizeof_ign(void) { return (int)sizeof(of_ign); }

/* ---- exact unit definitions used for the English-unit Rothermel chain (R16) */
#define M_PER_FT 0.3048
#define KG_PER_LB 0.45359237
#define J_PER_BTU 1055.05585262
#define MS_PER_FTMIN (M_PER_FT / 60.0)

/* latent heat of condensation of water, Sect. 2.3 (J/kg) */
#define L_COND 2.5e6

/*
 * The spread-rate chain of Sect. 2.2 / Table 2 for one (non-chaparral) fuel,
 * every intermediate kept.  The fuel data are first converted to English
 * units (Table 2 caption: lb, ft, min, BTU), then the table's rows are
 * evaluated in dependency order.  Readings where the table is garbled:
 * Gamma_max uses 0.0594 (R1); Q_ig = 250 + 1116 M_f (R2); beta_op =
 * 3.348 sigma^-0.8189 and B = 0.02526 sigma^0.54, Rothermel's definitions the
 * table uses without printing (R4); the moisture ratio is capped at 1 so
 * eta_M >= 0 (R15).  The wind and slope factors, which also depend on U and
 * tan(phi), are evaluated by the callers.
 */
typedef struct {
    double sigma, wl, delta, rhoP, h;           /* inputs in English units       */
    double w0, rhob, beta, beta_op, A, Gmax, Gamma, wn, etaM, etas, IR, xi, eps_h, Qig;
    double R0_ftmin;                            /* no-wind, no-slope rate, ft/min */
    double C, B, E;                             /* wind-factor constants          */
} rothermel;

static void rothermel_chain(const of_fuel *f, rothermel *o)
{
    double Mf = f->fuelmc_g;
    /* English units: lb/ft^2, ft, 1/ft, lb/ft^3, BTU/lb */
    o->wl = f->fgi * M_PER_FT * M_PER_FT / KG_PER_LB;
    o->delta = f->fueldepthm / M_PER_FT;
    o->sigma = f->savr * M_PER_FT;
    o->rhoP = f->fueldens * M_PER_FT * M_PER_FT * M_PER_FT / KG_PER_LB;
    o->h = f->cmbcnst * KG_PER_LB / J_PER_BTU;

    double sigma = o->sigma;
    o->w0 = o->wl / (1.0 + Mf);                      /* load net of moisture (CAWFE) */
    o->rhob = o->w0 / o->delta;                      /* oven-dry bulk density        */
    o->beta = o->rhob / o->rhoP;                     /* packing ratio                */
    o->beta_op = 3.348 * pow(sigma, -0.8189);        /* optimum packing ratio (R4)   */
    o->A = 1.0 / (4.77 * pow(sigma, 0.1) - 7.27);
    double s15 = pow(sigma, 1.5);
    o->Gmax = s15 / (495.0 + 0.0594 * s15);          /* (R1) */
    double rat = o->beta / o->beta_op;
    o->Gamma = o->Gmax * pow(rat, o->A) * exp(o->A * (1.0 - rat));
    o->wn = o->w0 / (1.0 + f->st);                   /* net of minerals */
    double r = Mf / f->fuelmce;
    if (r > 1.0) r = 1.0;                            /* (R15) */
    o->etaM = 1.0 - 2.59 * r + 5.11 * r * r - 3.52 * r * r * r;
    o->etas = 0.174 * pow(f->se, -0.19);
    o->IR = o->Gamma * o->wn * o->h * o->etaM * o->etas;   /* reaction intensity */
    o->xi = exp((0.792 + 0.681 * sqrt(sigma)) * (o->beta + 0.1)) / (192.0 + 0.2595 * sigma);
    o->eps_h = exp(-138.0 / sigma);                  /* effective heating number */
    o->Qig = 250.0 + 1116.0 * Mf;                    /* (R2) */
    o->R0_ftmin = o->IR * o->xi / (o->rhob * o->eps_h * o->Qig);

    o->C = 7.47 * exp(-0.133 * pow(sigma, 0.55));
    o->B = 0.02526 * pow(sigma, 0.54);               /* (R4) */
    o->E = 0.715 * exp(-3.59e-4 * sigma);
}

/*
 * Per-category spread-rate coefficients, Sect. 2.2 and Table 2.
 *
 * The no-wind rate R0 comes from the chain above, and the wind and slope
 * factors of Eq. (1) are folded into the coefficient form Eq. (3):
 *   R0*phi_W = c * U^b   with U the 6.1 m wind in m/s (clamped to [0, e]),
 *   R0*phi_S = d * tan^2(phi),
 * where phi_W = C (a U)^B (beta/beta_op)^(-E) with a U in ft/min (R3).
 * Chaparral (Eq. 2) is written in the coefficient form with S0 = 0.03333,
 * R0 = 0, b = 1, c = 1.2974, d = 0, e = 6/1.2974.
 *
 * Also tabulated: T_f from Eq. (4) (T_f = -600 w / (1000 ln 0.6) when tf<=0),
 * the sensible-flux factor w_l h/(1+M_f) of Eq. (5) and the latent factor
 * (M_f+0.56)/(1+M_f) L w_l of Eq. (6).
 */
int oracle_coef(const of_fuel *fu, int ncat, double wind_cap, double *tab)
{
    if (!fu || !tab || ncat <= 0) return -1;
    for (int k = 0; k < ncat; k++) {
        const of_fuel *f = &fu[k];
        double *row = tab + (size_t)k * OC_N;
        double Mf = f->fuelmc_g;

        row[OC_TF] = f->tf > 0.0 ? f->tf : -600.0 * f->weight / (1000.0 * log(0.6));
        row[OC_CH] = f->fgi * f->cmbcnst / (1.0 + Mf);
        row[OC_CQ] = (Mf + 0.56) / (1.0 + Mf) * L_COND * f->fgi;
        row[OC_M] = f->ros_mult;

        if (f->ichap) {
            row[OC_S0] = 0.03333;
            row[OC_R0] = 0.0;
            row[OC_B] = 1.0;
            row[OC_C] = 1.2974;
            row[OC_D] = 0.0;
            row[OC_E] = 6.0 / 1.2974;
            continue;
        }

        rothermel q;
        rothermel_chain(f, &q);
        double rat = q.beta / q.beta_op;
        double R0 = q.R0_ftmin * MS_PER_FTMIN;
        row[OC_S0] = 0.0;                               /* (R14) */
        row[OC_R0] = R0;
        row[OC_B] = q.B;
        /* R0*phi_W = R0*C*(beta/beta_op)^-E * (a*U/MS_PER_FTMIN)^B  (R3) */
        row[OC_C] = R0 * q.C * pow(rat, -q.E) * pow(f->windrf / MS_PER_FTMIN, q.B);
        row[OC_D] = R0 * 5.275 * pow(q.beta, -0.3);
        row[OC_E] = wind_cap;
    }
    return 0;
}

/* Intermediates of the chain as written out by oracle_rothermel_terms(). */
enum {
    ORT_SIGMA, ORT_WL, ORT_DELTA, ORT_RHOP, ORT_H, ORT_W0, ORT_RHOB, ORT_BETA, ORT_BETA_OP,
    ORT_A, ORT_GMAX, ORT_GAMMA, ORT_WN, ORT_ETAM, ORT_ETAS, ORT_IR, ORT_XI, ORT_EPS, ORT_QIG,
    ORT_R0_FTMIN, ORT_R0_MS, ORT_C, ORT_B, ORT_E, ORT_UA, ORT_PHIW, ORT_PHIS, ORT_S_MS, ORT_N
};

int oracle_nterms(void) { return ORT_N; }

/*
 * Product form Eq. (1), S = R0 (1 + phi_W + phi_S), with the wind factor
 * phi_W = C U_a^B (beta/beta_op)^(-E) (R3), U_a = a U in ft/min at midflame
 * (U clamped to [0, wind_cap], Table 2 caption), and the slope factor
 * phi_S = 5.275 beta^-0.3 tan^2(phi) (tan(phi) >= 0), evaluated directly
 * rather than through the coefficients.  Writes every intermediate of Table 2
 * (ORT_* order) to out[ORT_N] and returns ORT_N; the tests pin these values
 * against a hand evaluation of the printed formulas.  Chaparral fuels have no
 * chain (returns -1).
 */
int oracle_rothermel_terms(const of_fuel *f, double U, double tanphi, double wind_cap,
                           double *out)
{
    if (!f || !out || f->ichap) return -1;
    rothermel q;
    rothermel_chain(f, &q);
    double R0 = q.R0_ftmin;                                       /* ft/min */
    double Uc = fmin(wind_cap, fmax(0.0, U));                     /* m/s, clamped */
    double Ua = f->windrf * Uc / MS_PER_FTMIN;                    /* midflame ft/min */
    double phiW = q.C * pow(Ua, q.B) * pow(q.beta / q.beta_op, -q.E);
    double tp = fmax(0.0, tanphi);
    double phiS = 5.275 * pow(q.beta, -0.3) * tp * tp;
    out[ORT_SIGMA] = q.sigma;  out[ORT_WL] = q.wl;  out[ORT_DELTA] = q.delta;
    out[ORT_RHOP] = q.rhoP;  out[ORT_H] = q.h;  out[ORT_W0] = q.w0;  out[ORT_RHOB] = q.rhob;
    out[ORT_BETA] = q.beta;  out[ORT_BETA_OP] = q.beta_op;  out[ORT_A] = q.A;
    out[ORT_GMAX] = q.Gmax;  out[ORT_GAMMA] = q.Gamma;  out[ORT_WN] = q.wn;
    out[ORT_ETAM] = q.etaM;  out[ORT_ETAS] = q.etas;  out[ORT_IR] = q.IR;  out[ORT_XI] = q.xi;
    out[ORT_EPS] = q.eps_h;  out[ORT_QIG] = q.Qig;  out[ORT_R0_FTMIN] = R0;
    out[ORT_R0_MS] = R0 * MS_PER_FTMIN;
    out[ORT_C] = q.C;  out[ORT_B] = q.B;  out[ORT_E] = q.E;  out[ORT_UA] = Ua;
    out[ORT_PHIW] = phiW;  out[ORT_PHIS] = phiS;
    out[ORT_S_MS] = f->ros_mult * R0 * (1.0 + phiW + phiS) * MS_PER_FTMIN;
    return ORT_N;
}

/*
 * Product form Eq. (1) as a spread rate (m/s), with the per-category
 * multiplier; chaparral fuels use Eq. (2).  Only the tests call this: it pins
 * the coefficient form of Eq. (3).
 */
int oracle_ros_product(const of_fuel *f, double U, double tanphi, double wind_cap,
                       double *S_out)
{
    if (!f || !S_out) return -1;
    if (f->ichap) {                                      /* Eq. (2) */
        double s = 1.2974 * U;
        if (s < 0.03333) s = 0.03333;
        if (s > 6.0) s = 6.0;
        *S_out = s * f->ros_mult;
        return 0;
    }
    double t[ORT_N];
    oracle_rothermel_terms(f, U, tanphi, wind_cap, t);
    *S_out = t[ORT_S_MS];
    return 0;
}

/*
 * Spread rate in the coefficient form Eq. (3) with the per-category
 * multiplier m_k and the cap of reading R23:
 *   S = min{cap, m * max{S0, R0 + c min{e, max{0,U}}^b + d max{0,tan phi}^2}}.
 */
double oracle_ros(const double *row, double U, double tanphi, double ros_cap)
{
    double Uc = U > 0.0 ? U : 0.0;
    if (Uc > row[OC_E]) Uc = row[OC_E];
    double tp = tanphi > 0.0 ? tanphi : 0.0;
    double s = row[OC_R0] + row[OC_C] * pow(Uc, row[OC_B]) + row[OC_D] * tp * tp;
    if (s < row[OC_S0]) s = row[OC_S0];
    s = row[OC_M] * s;
    if (s > ros_cap) s = ros_cap;
    return s;
}

/*
 * Boundary extrapolation, Sect. 4.1: the ghost value beyond boundary node b
 * (with inner neighbour b1) is max{psi_b + (psi_b - psi_b1), psi_b, psi_b1}.
 */
static double ghost(double pb, double pb1)
{
    double lin = pb + (pb - pb1);
    double m = pb > pb1 ? pb : pb1;
    return lin > m ? lin : m;
}

/*
 * Copy psi[ny][nx] into ext[(ny+2)][(nx+2)] and fill one ghost layer.  The
 * y-ghost rows are filled first from the in-domain columns, then the x-ghost
 * columns for every row including the ghost rows, so a ghost corner is the x
 * extrapolation of the ghost row (reading R19; only the sub-cell quadrature
 * reads corners).  Needs nx >= 2 and ny >= 2.
 */
void oracle_extrapolate(const double *psi, int nx, int ny, double *ext)
{
    const int W = nx + 2;
#define EXT(i, j) ext[(size_t)((j) + 1) * W + ((i) + 1)]
#define PSI(i, j) psi[(size_t)(j) * nx + (i)]
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) EXT(i, j) = PSI(i, j);
    for (int i = 0; i < nx; i++) {
        EXT(i, -1) = ghost(PSI(i, 0), PSI(i, 1));
        EXT(i, ny) = ghost(PSI(i, ny - 1), PSI(i, ny - 2));
    }
    for (int j = -1; j <= ny; j++) {
        EXT(-1, j) = ghost(EXT(0, j), EXT(1, j));
        EXT(nx, j) = ghost(EXT(nx - 1, j), EXT(nx - 2, j));
    }
#undef EXT
#undef PSI
}

/*
 * Godunov upwind selection of Eq. (13) from the left and right one-sided
 * differences.  Overlapping cases are resolved first-match-wins in the
 * printed order (reading R12); the selected magnitude is the same either way.
 */
double oracle_godunov(double dm, double dp)
{
    if (dm <= 0.0 && dp <= 0.0) return dp;
    if (dm >= 0.0 && dp >= 0.0) return dm;
    if (dm <= 0.0 && dp >= 0.0) return 0.0;
    return fabs(dm) >= fabs(dp) ? dm : dp;
}

/*
 * Right-hand side F(psi) of Eq. (12) at every in-domain node, from the
 * extended array e (one ghost layer):
 *   F = -S(U.n, grad z.n) ||upwind grad psi|| + eps * [S] * Lap~ psi,
 * n from central differences of psi (Sect. 4.1, zero when the central
 * gradient vanishes, reading R13), the upwind gradient from Eq. (13) and the
 * dx-scaled five-point Laplacian Lap~.  viscosity_mode 0 multiplies the
 * viscous term by S (reading R9), mode 1 uses the literal eps*Lap~.
 */
static void rhs(const of_mesh *m, const double *tab, const uint8_t *cat,
                const double *gzx, const double *gzy, const double *u, const double *v,
                const of_prm *p, const double *e, double *F)
{
    const int nx = m->nx, ny = m->ny, W = nx + 2;
    const double dx = m->dx, dy = m->dy;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            size_t c0 = (size_t)(j + 1) * W + (i + 1);
            double pc = e[c0], pw = e[c0 - 1], pe = e[c0 + 1];
            double ps = e[c0 - W], pn = e[c0 + W];
            size_t k = (size_t)j * nx + i;

            double gx = oracle_godunov((pc - pw) / dx, (pe - pc) / dx);
            double gy = oracle_godunov((pc - ps) / dy, (pn - pc) / dy);
            double up_norm = sqrt(gx * gx + gy * gy);

            double cx = (pe - pw) / (2.0 * dx);
            double cy = (pn - ps) / (2.0 * dy);
            double cn = sqrt(cx * cx + cy * cy);
            double nxv = 0.0, nyv = 0.0;
            if (cn > 0.0) { nxv = cx / cn; nyv = cy / cn; }

            double Un = u[k] * nxv + v[k] * nyv;          /* U = U.n       */
            double tn = gzx[k] * nxv + gzy[k] * nyv;      /* tan phi = grad z.n */
            double S = oracle_ros(tab + (size_t)cat[k] * OC_N, Un, tn, p->ros_cap);

            double lap = (pe - 2.0 * pc + pw) / dx + (pn - 2.0 * pc + ps) / dy;
            double visc = p->viscosity_mode == 0 ? p->viscosity * S * lap
                                                 : p->viscosity * lap;
            F[k] = -S * up_norm + visc;
        }
    }
}

/* Distance from (x,y) to the segment a-b, and the arc length from a to the
 * nearest point (for the drip torch). */
static double seg_dist(double x, double y, double ax, double ay, double bx, double by,
                       double *along)
{
    double dxs = bx - ax, dys = by - ay;
    double L2 = dxs * dxs + dys * dys;
    double s = 0.0;
    if (L2 > 0.0) {
        s = ((x - ax) * dxs + (y - ay) * dys) / L2;
        if (s < 0.0) s = 0.0;
        if (s > 1.0) s = 1.0;
    }
    double qx = ax + s * dxs, qy = ay + s * dys;
    if (along) *along = s * sqrt(L2);
    return sqrt((x - qx) * (x - qx) + (y - qy) * (y - qy));
}

/*
 * Whether ignition g is active at the start of the step at time t, Sect. 4.4:
 * t_g <= t <= t_g + r_g/S_g for a segment, t_g <= t <= t_h + r_g/S_g for a
 * drip torch (S_g = inf gives r_g/S_g = 0).
 */
int oracle_ign_active(const of_ign *g, double t)
{
    int torch = (g->vx != 0.0 || g->vy != 0.0);
    double tend = torch ? g->t_end : g->t_start;
    double grow = isinf(g->ros) ? 0.0 : g->radius / g->ros;
    return t >= g->t_start && t <= tend + grow;
}

/*
 * Level set of the initial fire of ignition g at point (x,y) and time t,
 * Eq. (20) and its drip-torch form: dist(x, segment(t)) - min{r_g, S_g(t-t_g)},
 * with the radius r_g at once when S_g = inf (reading R18).  *arrive gets the
 * arrival time of the initial fire at (x,y): the time the segment point
 * nearest to (x,y) was laid down plus dist/S_g, capped at t (reading R18).
 */
double oracle_ign_psi(const of_ign *g, double x, double y, double t, double *arrive)
{
    int torch = (g->vx != 0.0 || g->vy != 0.0);
    double bx = g->bx, by = g->by;
    if (torch) {
        double te = t < g->t_end ? t : g->t_end;
        bx = g->ax + g->vx * (te - g->t_start);
        by = g->ay + g->vy * (te - g->t_start);
    }
    double along = 0.0;
    double d = seg_dist(x, y, g->ax, g->ay, bx, by, &along);
    double rad = isinf(g->ros) ? g->radius : fmin(g->radius, g->ros * (t - g->t_start));
    if (arrive) {
        double tlay = g->t_start;
        if (torch) tlay += along / sqrt(g->vx * g->vx + g->vy * g->vy);
        double a = isinf(g->ros) ? tlay : tlay + d / g->ros;
        *arrive = a < t ? a : t;
    }
    return d - rad;
}

/*
 * Step 1 of Sect. 6, ignition (Sect. 4.4, Eq. 21): psi := min{psi, psi_g} for
 * every active ignition; a node that goes from psi > 0 to psi <= 0 with no
 * ignition time yet gets the earliest arrival time among the ignitions that
 * cover it (reading R18).
 */
static void ignite(const of_mesh *m, const of_ign *ign, int nign, double t,
                   double *psi, double *tign)
{
    int any = 0;
    for (int g = 0; g < nign; g++) any |= oracle_ign_active(&ign[g], t);
    if (!any) return;
    const int nx = m->nx, ny = m->ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            size_t k = (size_t)j * nx + i;
            double x = (i + 0.5) * m->dx, y = (j + 0.5) * m->dy;
            double pold = psi[k], pnew = pold, tarr = INFINITY;
            for (int g = 0; g < nign; g++) {
                if (!oracle_ign_active(&ign[g], t)) continue;
                double a;
                double pg = oracle_ign_psi(&ign[g], x, y, t, &a);
                if (pg < pnew) pnew = pg;
                if (pg <= 0.0 && a < tarr) tarr = a;
            }
            psi[k] = pnew;
            if (pold > 0.0 && pnew <= 0.0 && isinf(tign[k])) tign[k] = tarr;
        }
    }
}

/*
 * Burned fraction of one sub-cell, Eqs. (18)-(19):
 *   beta = (1 - sum psi_k / sum |psi_k|)/2   (0 when all psi_k = 0, R11),
 *   burned = beta * (1 - exp(-(1/4) sum (t - t_k)/T_f)),
 * with t_k already replaced by t where psi_k >= 0 (Eq. 17, reading R10) and
 * the sign of the exponent read as in Eq. (4) (reading R8).
 */
double oracle_subcell_beta(const double *psi4)
{
    double s = 0.0, a = 0.0;
    for (int k = 0; k < 4; k++) { s += psi4[k]; a += fabs(psi4[k]); }
    return a > 0.0 ? 0.5 * (1.0 - s / a) : 0.0;
}

double oracle_subcell_burned(const double *psi4, const double *ti4, double t, double Tf)
{
    double beta = oracle_subcell_beta(psi4);
    double tau = 0.0;
    for (int k = 0; k < 4; k++) tau += (t - ti4[k]) / Tf;
    tau *= 0.25;
    return beta * (1.0 - exp(-tau));
}

/*
 * Fuel fraction of one cell, Eqs. (15)-(19) and Fig. 2, from the 3x3 block of
 * node values centred on the cell (row-major, [dy+1][dx+1] for dx,dy in
 * -1..1): psi and the node ignition time t^ (already t where psi >= 0).  The
 * cell splits into four sub-cells whose corners are the cell centre, two edge
 * midpoints and one cell corner; psi and t^ are interpolated bilinearly to
 * those points and t^ is reset to t where the interpolated psi >= 0.
 *   F = 1 - (1/4) sum_subcells burned.
 */
double oracle_cell_frac(const double *p9, const double *t9, double t, double Tf)
{
#define P(a, b) p9[((b) + 1) * 3 + ((a) + 1)]
#define T(a, b) t9[((b) + 1) * 3 + ((a) + 1)]
    double burned = 0.0;
    for (int sb = -1; sb <= 1; sb += 2) {
        for (int sa = -1; sa <= 1; sa += 2) {
            double ps[4], ts[4];
            /* centre */
            ps[0] = P(0, 0);
            ts[0] = T(0, 0);
            /* midpoint of the x edge */
            ps[1] = 0.5 * (P(0, 0) + P(sa, 0));
            ts[1] = 0.5 * (T(0, 0) + T(sa, 0));
            /* midpoint of the y edge */
            ps[2] = 0.5 * (P(0, 0) + P(0, sb));
            ts[2] = 0.5 * (T(0, 0) + T(0, sb));
            /* cell corner */
            ps[3] = 0.25 * (P(0, 0) + P(sa, 0) + P(0, sb) + P(sa, sb));
            ts[3] = 0.25 * (T(0, 0) + T(sa, 0) + T(0, sb) + T(sa, sb));
            for (int k = 0; k < 4; k++)
                if (ps[k] >= 0.0) ts[k] = t;      /* Eq. (17) at the sub-cell corners */
            burned += oracle_subcell_burned(ps, ts, t, Tf);
        }
    }
    return 1.0 - 0.25 * burned;
#undef P
#undef T
}

/*
 * One fire-model time step from time t to t + dt, Sect. 6 steps 1-6 and the
 * boundary check of Sect. 4.1.  psi, tign, frac are [ny][nx] and are updated
 * in place; fsens, flat are [ceil(ny/sr_y)][ceil(nx/sr_x)] outputs (W/m^2);
 * status gets OS_BOUNDARY / OS_NONFINITE bits OR-ed in.
 */
int oracle_step(const of_mesh *m, const double *tab, int ncat, const uint8_t *cat,
                const double *gzx, const double *gzy, const double *u, const double *v,
                const of_ign *ign, int nign, const of_prm *p, double t, double dt,
                double *psi, double *tign, double *frac, double *fsens, double *flat,
                int32_t *status)
{
    const int nx = m->nx, ny = m->ny;
    if (nx < 2 || ny < 2 || m->sr_x < 1 || m->sr_y < 1 || !(dt > 0.0)) return -1;
    const size_t n = (size_t)nx * ny, ne = (size_t)(nx + 2) * (ny + 2);
    for (size_t k = 0; k < n; k++)
        if (cat[k] >= ncat) return -1;

    double *ext = (double *)malloc(ne * sizeof(double));
    double *F1 = (double *)malloc(n * sizeof(double));
    double *F2 = (double *)malloc(n * sizeof(double));
    double *ps = (double *)malloc(n * sizeof(double));
    double *p0 = (double *)malloc(n * sizeof(double));
    double *tex = (double *)malloc(ne * sizeof(double));
    double *fnew = (double *)malloc(n * sizeof(double));
    if (!ext || !F1 || !F2 || !ps || !p0 || !tex || !fnew) {
        free(ext); free(F1); free(F2); free(ps); free(p0); free(tex); free(fnew);
        return -2;
    }

    /* (1) ignition at the start of the step */
    ignite(m, ign, nign, t, psi, tign);
    memcpy(p0, psi, n * sizeof(double));

    /* (2) Heun's method, Eq. (11), with the ghost layer re-extrapolated for
     * each stage (Sect. 4.1) */
    oracle_extrapolate(p0, nx, ny, ext);
    rhs(m, tab, cat, gzx, gzy, u, v, p, ext, F1);
    for (size_t k = 0; k < n; k++) ps[k] = p0[k] + dt * F1[k];
    oracle_extrapolate(ps, nx, ny, ext);
    rhs(m, tab, cat, gzx, gzy, u, v, p, ext, F2);
    for (size_t k = 0; k < n; k++) psi[k] = p0[k] + dt * (0.5 * F1[k] + 0.5 * F2[k]);

    /* (3) ignition time of nodes crossed during the step, Eq. (14); the first
     * crossing is kept (reading R18) */
    for (size_t k = 0; k < n; k++) {
        if (p0[k] > 0.0 && psi[k] <= 0.0 && isinf(tign[k]))
            tign[k] = t + p0[k] * dt / (p0[k] - psi[k]);
    }

    /* (4) fuel fraction at t' = t + dt, Sect. 4.3 */
    const double tp = t + dt;
    oracle_extrapolate(psi, nx, ny, ext);
    {
        const int W = nx + 2;
        for (size_t k = 0; k < ne; k++) tex[k] = tp;             /* ghost nodes: t' (R19) */
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t k = (size_t)j * nx + i;
                tex[(size_t)(j + 1) * W + (i + 1)] = psi[k] >= 0.0 ? tp : tign[k];  /* Eq. (17) */
            }
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; j++) {
            for (int i = 0; i < nx; i++) {
                double p9[9], t9[9];
                for (int b = -1; b <= 1; b++)
                    for (int a = -1; a <= 1; a++) {
                        size_t q = (size_t)(j + 1 + b) * W + (i + 1 + a);
                        p9[(b + 1) * 3 + (a + 1)] = ext[q];
                        t9[(b + 1) * 3 + (a + 1)] = tex[q];
                    }
                size_t k = (size_t)j * nx + i;
                fnew[k] = oracle_cell_frac(p9, t9, tp, tab[(size_t)cat[k] * OC_N + OC_TF]);
            }
        }
    }

    /* (5) per-cell flux densities, Eqs. (5)-(6), and (6) their mean over the
     * fire cells of each atmosphere cell (partial cells at the far edges
     * average over the fire cells they contain, reading R20) */
    const int nax = (nx + m->sr_x - 1) / m->sr_x, nay = (ny + m->sr_y - 1) / m->sr_y;
#pragma omp parallel for schedule(static)
    for (int J = 0; J < nay; J++) {
        for (int I = 0; I < nax; I++) {
            double ssum = 0.0, lsum = 0.0;
            int cnt = 0;
            for (int j = J * m->sr_y; j < (J + 1) * m->sr_y && j < ny; j++)
                for (int i = I * m->sr_x; i < (I + 1) * m->sr_x && i < nx; i++) {
                    size_t k = (size_t)j * nx + i;
                    const double *row = tab + (size_t)cat[k] * OC_N;
                    double dF = (frac[k] - fnew[k]) / dt;
                    ssum += dF * row[OC_CH];
                    lsum += dF * row[OC_CQ];
                    cnt++;
                }
            fsens[(size_t)J * nax + I] = ssum / cnt;
            flat[(size_t)J * nax + I] = lsum / cnt;
        }
    }
    memcpy(frac, fnew, n * sizeof(double));

    /* boundary check, Sect. 4.1: fire in the guard ring ends the run */
    int32_t st = 0;
    const int gw = p->guard_width;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t k = (size_t)j * nx + i;
            int edge = i < gw || j < gw || i >= nx - gw || j >= ny - gw;
            if (edge && psi[k] < 0.0) st |= OS_BOUNDARY;
            if (!isfinite(psi[k]) || !isfinite(frac[k])) st |= OS_NONFINITE;
        }
    *status |= st;

    free(ext); free(F1); free(F2); free(ps); free(p0); free(tex); free(fnew);
    return 0;
}
