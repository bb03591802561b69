/*
 * odust_oracle.c -- plain, slow FP64 CPU oracle of the dust-in-ion-flow step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header or constant table with the HIP
 * library: it works in SI units and FP64 throughout, follows the paper's
 * formulas term by term, and parallelises only the outer ion loop with
 * OpenMP (each ion's sum runs over j in increasing order, so results do not
 * depend on the thread count).
 *
 * Paper: Kolotinskii & Timofeev, "OpenDust: A fast GPU-accelerated code for
 * calculation forces, acting on microparticles in a plasma flow"
 * (arXiv 2205.06557).  Sections cited below:
 *   Sec. 2 (Methods)        -- superparticles, Boltzmann electrons (screened
 *                              ion-ion force), asymmetric ion-dust model,
 *                              velocity-Verlet push, constant-frequency
 *                              charge exchange, open boundary, Eqs. (1)-(4),
 *                              the three charging models.
 *   Sec. 3                  -- parameter objects (SI units), observables.
 *   Appendix B, Eqs. (B.1)-(B.12) -- flux-conserving reinjection.
 * Where the paper is silent the reading taken is stated at the function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 exact / recommended values. */
#define ORC_QE   1.602176634e-19     /* C      */
#define ORC_KB   1.380649e-23        /* J/K    */
#define ORC_EPS0 8.8541878128e-12    /* F/m    */
#define ORC_ME   9.1093837015e-31    /* kg     */
#define ORC_PI   3.14159265358979323846

#define ORC_MAXD 64

/* Philox purposes (counter word 2). */
#define ORC_P_INIT_POS 0
#define ORC_P_INIT_VEL 1
#define ORC_P_COLL     2
#define ORC_P_REINJ    3

/* flags */
#define ORC_F_LITERAL_SIDE 1u   /* side injection: radial + v_z only (Eqs. B.10-B.11 literally) */
#define ORC_F_NO_ION_ION   2u   /* test-particle mode: ion-ion force off */
#define ORC_F_FIELD_DRIVEN 8u   /* field-driven collisional flow: injection and initial v_z
                                   from the stationary distribution of the drift between
                                   charge-exchange collisions (needs nu > 0) */
#define ORC_F_CONFINEMENT  4u   /* confinement field of the outer plasma (Appendix A); the
                                   driver fits it after orc_init and installs it with
                                   orc_set_confinement */

/* event codes per ion for the last step */
#define ORC_EV_NONE   (-1)
#define ORC_EV_EXITED (-2)

typedef struct orc_sys {
    /* inputs (SI) */
    double Te, Ti, n, mi, mach, nu, E_in;
    double R, H, dt;
    int64_t N, n_discard;
    uint64_t seed, sysid;
    int mode, flags, nd;
    double dpos[ORC_MAXD][3], da[ORC_MAXD], dq0[ORC_MAXD];
    /* derived */
    double lam, wpi, cs, sig, u, V, w, q, m, E, Pc;
    double ufd;             /* field-driven flow: mean drift gained between collisions, eE/(m nu) */
    double Jb, Jt, Js;
    uint64_t Tc, Tb, Tbt;
    /* state */
    double *x, *v;          /* [N][3] */
    double Q[ORC_MAXD];     /* C */
    int64_t step;
    /* outputs of the last step */
    double *a;              /* [N][3], accelerations at x^n */
    int32_t *ev;            /* per ion event code */
    int32_t *hit;           /* per ion: 1 if a charge-exchange collision happened */
    double Qrec[ORC_MAXD];
    double F[ORC_MAXD][4][3];
    int64_t nabs[ORC_MAXD], nexit, ncoll;
    /* running averages over recorded steps n >= n_discard */
    double sumQ[ORC_MAXD], sumF[ORC_MAXD][4][3];
    int64_t nrec;
    int status;
    /* confinement field of the outer plasma (Appendix A): fitted polynomial
     * P(r, z) = sum_m alpha_m (r/rs)^(2 a_m) (z/zs)^(2 b_m), in volts */
    int conf_on;
    double conf_alpha[15], conf_rs, conf_zs;
    /* ion-ion cutoff with a switching function (Section 4, performance with
     * cutoff): r_sw < r_cut in m, cut_on = 0 for the plain all-pairs sum */
    int cut_on;
    double r_sw, r_cut;
} orc_sys;

/* Exponent pairs (a, b) of the fifteen terms r^(2a) z^(2b) of Eq. (A.3), in
 * the order alpha_0 .. alpha_14. */
static const int ORC_PA[15] = {0, 1, 0, 1, 2, 0, 2, 1, 3, 0, 2, 3, 1, 4, 0};
static const int ORC_PB[15] = {0, 0, 1, 1, 0, 2, 1, 2, 0, 3, 2, 1, 3, 0, 4};

static double orc_ipow(double x, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

/* Confinement field E_out = -grad P (Eq. (A.4)) at x (SI, V/m). */
static void orc_confinement_field(const orc_sys* s, const double x[3], double E[3])
{
    double u = (x[0] * x[0] + x[1] * x[1]) / (s->conf_rs * s->conf_rs);
    double v = x[2] * x[2] / (s->conf_zs * s->conf_zs);
    double dPdu = 0.0, dPdv = 0.0;   /* derivatives with respect to u and v */
    for (int m = 0; m < 15; ++m) {
        int a = ORC_PA[m], b = ORC_PB[m];
        if (a > 0) dPdu += s->conf_alpha[m] * a * orc_ipow(u, a - 1) * orc_ipow(v, b);
        if (b > 0) dPdv += s->conf_alpha[m] * b * orc_ipow(u, a) * orc_ipow(v, b - 1);
    }
    /* dP/dx = dP/du * 2x/rs^2, dP/dz = dP/dv * 2z/zs^2 */
    E[0] = -dPdu * 2.0 * x[0] / (s->conf_rs * s->conf_rs);
    E[1] = -dPdu * 2.0 * x[1] / (s->conf_rs * s->conf_rs);
    E[2] = -dPdv * 2.0 * x[2] / (s->conf_zs * s->conf_zs);
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11), written from the
 * published round description: two 64x64->128 multiplies per round, the
 * high halves xored with the other two words and the key, key bumped by the
 * Weyl constants between rounds.                                            */
static void orc_mulhilo(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        uint64_t h0, l0, h1, l1;
        orc_mulhilo(0xD2E7470EE14C6C93ULL, c0, &h0, &l0);
        orc_mulhilo(0xCA5A826395121157ULL, c2, &h1, &l1);
        uint64_t n0 = h1 ^ c1 ^ k0;
        uint64_t n2 = h0 ^ c3 ^ k1;
        c0 = n0; c1 = l1; c2 = n2; c3 = l0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void orc_draw(const orc_sys* s, uint64_t ion, uint64_t stepn, uint64_t purpose,
                     uint64_t sub, uint64_t w[4])
{
    uint64_t ctr[4] = {ion, stepn, purpose, sub};
    uint64_t key[2] = {s->seed, s->sysid};
    orc_philox(ctr, key, w);
}

/* Uniform strictly inside (0,1): the top 52 bits plus one half, times 2^-52
 * (exact in FP64: k + 1/2 with k < 2^52 fits the 53-bit significand). */
double orc_uniform(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * (1.0 / 4503599627370496.0);
}

/* Box-Muller pair from two uniforms. */
static void orc_box_muller(double ua, double ub, double* g1, double* g2)
{
    double rad = sqrt(-2.0 * log(ua));
    *g1 = rad * cos(2.0 * ORC_PI * ub);
    *g2 = rad * sin(2.0 * ORC_PI * ub);
}

/* ------------------------------------------------------------------------ */
/* Standard normal pdf / tails. */
static double orc_pdf(double t) { return exp(-0.5 * t * t) / sqrt(2.0 * ORC_PI); }
static double orc_Phi(double t) { return 0.5 * erfc(-t / sqrt(2.0)); }
static double orc_Phic(double t) { return 0.5 * erfc(t / sqrt(2.0)); }

/* Integral inflow through a flat face for a normal N(ubar, sig^2) velocity
 * distribution along the face normal, per unit area: int_0^inf v phi(v) dv
 * (Eqs. B.2-B.3 with the shifted Maxwellian of Eq. B.1). */
double orc_face_flux(double ubar, double sig)
{
    return ubar * orc_Phi(ubar / sig) + sig * orc_pdf(ubar / sig);
}

/* Tail of the flux-weighted distribution: int_v^inf v' phi(v') dv' for
 * v >= 0, phi = N(ubar, sig^2).  The cumulative distributions G_bottom and
 * G_top of Eqs. (B.8)-(B.9) are (total - tail). */
double orc_flux_tail(double v, double ubar, double sig)
{
    double t = (v - ubar) / sig;
    return ubar * orc_Phic(t) + sig * orc_pdf(t);
}

/* Inverse of the flux-weighted velocity distribution on v >= 0: the v with
 * G(v) = (1-uu) G(inf), i.e. tail(v) = uu * G(inf).  Safeguarded Newton
 * (tail'(v) = -v phi(v)) with bisection fallback on [0, max(ubar,0)+40 sig],
 * stopped at |dv| <= 1e-13 sig.  At ubar = 0 this is sig*sqrt(-2 ln uu). */
double orc_flux_inverse(double uu, double ubar, double sig)
{
    double total = orc_face_flux(ubar, sig);
    double target = uu * total;
    double lo = 0.0, hi = (ubar > 0.0 ? ubar : 0.0) + 40.0 * sig;
    double v = (ubar > 0.0 ? ubar : 0.0) + sig;
    for (int it = 0; it < 400; ++it) {
        double g = orc_flux_tail(v, ubar, sig) - target;   /* decreasing in v */
        if (g > 0.0) lo = v; else hi = v;
        double slope = -v * orc_pdf((v - ubar) / sig) / sig;
        double vn;
        if (slope < 0.0) {
            vn = v - g / slope;
            if (!(vn > lo && vn < hi)) vn = 0.5 * (lo + hi);
        } else {
            vn = 0.5 * (lo + hi);
        }
        if (fabs(vn - v) <= 1e-13 * sig) { v = vn; break; }
        v = vn;
    }
    return v;
}

/* ------------------------------------------------------------------------ */
/* Field-driven collisional flow (Section 2: homogeneous driving field,
 * charge exchange at constant frequency nu that restarts an ion from the
 * neutrals' Maxwellian).  Between collisions an ion gains a t along z, and in
 * a stationary flow the time since the last collision is exponential with
 * rate nu, so v_z = sig g + ufd T with g ~ N(0,1), T ~ Exp(1), ufd = a/nu:
 * the Gaussian convolved with an exponential, the phi(v_z) of Eq. (B.1) for
 * this flow (v_x, v_y stay Maxwellian).  With A(x) = exp(c - x/ufd)
 * Phi(x/sig - sig/ufd), c = sig^2/(2 ufd^2):
 *   phi(x)                         = A(x) / ufd,
 *   int_x^inf v phi(v) dv          = (x + ufd) A(x) + sig pdf(x/sig) + ufd Phic(x/sig),
 *   -int_-inf^(-w) v phi(v) dv     = (ufd - w) A(-w) + sig pdf(w/sig) - ufd Phic(w/sig),
 * obtained by integrating by parts (the exponential factors of A combine
 * with the Gaussian into pdf(x/sig)).  Valid for sig/ufd up to about 30. */
static double orc_fd_A(double x, double ufd, double sig)
{
    double c = 0.5 * sig * sig / (ufd * ufd);
    return exp(c - x / ufd) * orc_Phi(x / sig - sig / ufd);
}

double orc_fd_density(double x, double ufd, double sig) { return orc_fd_A(x, ufd, sig) / ufd; }

/* int_x^inf v phi(v) dv; at x = 0 the inflow per unit area of the bottom face */
double orc_fd_tail(double x, double ufd, double sig)
{
    return (x + ufd) * orc_fd_A(x, ufd, sig) + sig * orc_pdf(x / sig) + ufd * orc_Phic(x / sig);
}

/* -int_-inf^(-w) v phi(v) dv for w >= 0; at w = 0 the inflow of the top face */
double orc_fd_head(double w, double ufd, double sig)
{
    return (ufd - w) * orc_fd_A(-w, ufd, sig) + sig * orc_pdf(w / sig) - ufd * orc_Phic(w / sig);
}

/* Flux-weighted inward speed at a face (Eqs. (B.8)-(B.9) with the
 * field-driven phi): the s >= 0 with tail(s) = uu * tail(0), where tail is
 * orc_fd_tail (bottom, v_z = s) or orc_fd_head (top, v_z = -s).  Bisection
 * on [0, 40 sig + 50 ufd] to |ds| <= 1e-13 sig. */
double orc_fd_inverse(double uu, double ufd, double sig, int top)
{
    double target = uu * (top ? orc_fd_head(0.0, ufd, sig) : orc_fd_tail(0.0, ufd, sig));
    double lo = 0.0, hi = 40.0 * sig + (top ? 0.0 : 50.0 * ufd);
    while (hi - lo > 1e-13 * sig) {
        double mid = 0.5 * (lo + hi);
        double t = top ? orc_fd_head(mid, ufd, sig) : orc_fd_tail(mid, ufd, sig);
        if (t > target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* OML currents (Section 2, charging models; Allen 1992).
 * Electron current: Boltzmann-repelled random flux for phi < 0, OML-attracted
 * for phi >= 0.  Ion current: OML cross-section pi a^2 (1 - 2 e phi/(m v^2))
 * averaged over the drifting Maxwellian N((0,0,u), sig^2 I).  Both in A. */
double orc_electron_current(double Q, double a, double n, double Te)
{
    double phi = Q / (4.0 * ORC_PI * ORC_EPS0 * a);
    double vth = sqrt(8.0 * ORC_KB * Te / (ORC_PI * ORC_ME));
    double x = ORC_QE * phi / (ORC_KB * Te);
    double fac = (phi < 0.0) ? exp(x) : (1.0 + x);
    return -ORC_PI * a * a * n * ORC_QE * vth * fac;
}

double orc_ion_current_oml(double Q, double a, double n, double Ti, double mi, double u)
{
    double phi = Q / (4.0 * ORC_PI * ORC_EPS0 * a);
    double chi = (phi < 0.0) ? -ORC_QE * phi / (ORC_KB * Ti) : 0.0;
    double vt = sqrt(2.0 * ORC_KB * Ti / mi);
    double s = u / vt;
    double bracket;
    if (s < 1e-6)
        bracket = (2.0 / sqrt(ORC_PI)) * (1.0 + chi);
    else
        bracket = exp(-s * s) / sqrt(ORC_PI) + (s * s + 0.5 + chi) * erf(s) / s;
    return ORC_PI * a * a * n * ORC_QE * vt * bracket;
}

/* ------------------------------------------------------------------------ */
/* Derived quantities.
 *   lambda = r_De, omega_pi, c_s = sqrt(kB Te/mi), sigma = sqrt(kB Ti/mi);
 *   flow u = M c_s (Mach measured against c_s);
 *   superparticle weight w = n V / N: charge q = w e, mass m = w mi
 *     (same q/m as an ion, Section 2);
 *   driving field: given, or mi nu u / e when not given and nu > 0
 *     (steady drift eE/(mi nu) = u);
 *   charge-exchange probability per step P_c = 1 - exp(-nu dt);
 *   face inflows J (Eqs. B.2-B.4 in closed form), probabilities (B.5-B.7). */
static uint64_t orc_prob_to_u64(double p)
{
    if (!(p > 0.0)) return 0;
    double t = p * 18446744073709551616.0;
    if (t >= 18446744073709551615.0) return UINT64_MAX;
    return (uint64_t)t;
}

static void orc_derive(orc_sys* s)
{
    s->lam = sqrt(ORC_EPS0 * ORC_KB * s->Te / (s->n * ORC_QE * ORC_QE));
    s->wpi = sqrt(s->n * ORC_QE * ORC_QE / (ORC_EPS0 * s->mi));
    s->cs = sqrt(ORC_KB * s->Te / s->mi);
    s->sig = sqrt(ORC_KB * s->Ti / s->mi);
    s->u = s->mach * s->cs;
    s->V = ORC_PI * s->R * s->R * s->H;
    s->w = s->n * s->V / (double)s->N;
    s->q = s->w * ORC_QE;
    s->m = s->w * s->mi;
    if (isnan(s->E_in))
        s->E = (s->nu > 0.0) ? s->mi * s->nu * s->u / ORC_QE : 0.0;
    else
        s->E = s->E_in;
    s->Pc = -expm1(-s->nu * s->dt);
    s->Tc = orc_prob_to_u64(s->Pc);
    s->ufd = (s->nu > 0.0) ? ORC_QE * s->E / (s->mi * s->nu) : 0.0;
    if (s->flags & ORC_F_FIELD_DRIVEN) {
        s->Jb = ORC_PI * s->R * s->R * orc_fd_tail(0.0, s->ufd, s->sig);
        s->Jt = ORC_PI * s->R * s->R * orc_fd_head(0.0, s->ufd, s->sig);
    } else {
        s->Jb = ORC_PI * s->R * s->R * orc_face_flux(s->u, s->sig);
        s->Jt = ORC_PI * s->R * s->R * orc_face_flux(-s->u, s->sig);
    }
    s->Js = 2.0 * ORC_PI * s->R * s->H * s->sig / sqrt(2.0 * ORC_PI);
    double J = s->Jb + s->Jt + s->Js;
    s->Tb = orc_prob_to_u64(s->Jb / J);
    s->Tbt = orc_prob_to_u64((s->Jb + s->Jt) / J);
}

/* ------------------------------------------------------------------------ */
orc_sys* orc_create(const double* plasma /*Te,Ti,n,mi,mach,nu,E*/,
                    const double* geom /*R,H,dt*/,
                    int64_t N, int64_t n_discard, uint64_t seed, uint64_t sysid,
                    int mode, int flags, const double* dust /*[nd][5] x,y,z,a,q0*/, int nd)
{
    if (N < 1 || nd < 0 || nd > ORC_MAXD) return NULL;
    if ((flags & ORC_F_FIELD_DRIVEN) && !(plasma[5] > 0.0)) return NULL;
    orc_sys* s = (orc_sys*)calloc(1, sizeof(orc_sys));
    if (!s) return NULL;
    s->Te = plasma[0]; s->Ti = plasma[1]; s->n = plasma[2]; s->mi = plasma[3];
    s->mach = plasma[4]; s->nu = plasma[5]; s->E_in = plasma[6];
    s->R = geom[0]; s->H = geom[1]; s->dt = geom[2];
    s->N = N; s->n_discard = n_discard; s->seed = seed; s->sysid = sysid;
    s->mode = mode; s->flags = flags; s->nd = nd;
    for (int d = 0; d < nd; ++d) {
        s->dpos[d][0] = dust[5 * d + 0];
        s->dpos[d][1] = dust[5 * d + 1];
        s->dpos[d][2] = dust[5 * d + 2];
        s->da[d] = dust[5 * d + 3];
        s->dq0[d] = dust[5 * d + 4];
    }
    orc_derive(s);
    s->x = (double*)calloc((size_t)N * 3, sizeof(double));
    s->v = (double*)calloc((size_t)N * 3, sizeof(double));
    s->a = (double*)calloc((size_t)N * 3, sizeof(double));
    s->ev = (int32_t*)calloc((size_t)N, sizeof(int32_t));
    s->hit = (int32_t*)calloc((size_t)N, sizeof(int32_t));
    if (!s->x || !s->v || !s->a || !s->ev || !s->hit) {
        free(s->x); free(s->v); free(s->a); free(s->ev); free(s->hit); free(s);
        return NULL;
    }
    for (int d = 0; d < nd; ++d) s->Q[d] = s->dq0[d];
    return s;
}

void orc_destroy(orc_sys* s)
{
    if (!s) return;
    free(s->x); free(s->v); free(s->a); free(s->ev); free(s->hit);
    free(s);
}

/* Derived constants, for tests: lam, wpi, cs, sig, u, V, w, q, m, E, Pc,
 * Jb, Jt, Js, ufd (15 doubles) and Tc, Tb, Tbt (3 uint64). */
void orc_derived(const orc_sys* s, double* d15, uint64_t* t3)
{
    double d[15] = {s->lam, s->wpi, s->cs, s->sig, s->u, s->V, s->w, s->q, s->m,
                    s->E, s->Pc, s->Jb, s->Jt, s->Js, s->ufd};
    memcpy(d15, d, sizeof d);
    t3[0] = s->Tc; t3[1] = s->Tb; t3[2] = s->Tbt;
}

static int orc_inside_grain(const orc_sys* s, const double p[3])
{
    for (int d = 0; d < s->nd; ++d) {
        double dx = p[0] - s->dpos[d][0], dy = p[1] - s->dpos[d][1], dz = p[2] - s->dpos[d][2];
        if (dx * dx + dy * dy + dz * dz <= s->da[d] * s->da[d]) return 1;
    }
    return 0;
}

/* Initial state (Section 2: homogeneous plasma flowing with a shifted
 * Maxwellian).  Ion i: attempt k uses block (i, 0, INIT_POS, k) and takes
 * r = R sqrt(u0), theta = 2 pi u1, z = H (u2 - 1/2); the first attempt
 * outside every grain is kept.  Velocity from block (i, 0, INIT_VEL, 0):
 * normals (g1,g2) from (u0,u1), g3 from (u2,u3); v = (sig g1, sig g2,
 * u + sig g3), taken as the half-step velocity v^{-1/2}.  Field-driven flow:
 * v_z = sig g3 + ufd T instead, T = -ln u0 of block (i, 0, INIT_VEL, 1).
 * Q_d = q0_d. */
int orc_init(orc_sys* s)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int64_t i = 0; i < s->N; ++i) {
        double p[3];
        int ok = 0;
        for (uint64_t k = 0; k < 1000; ++k) {
            uint64_t w[4];
            orc_draw(s, (uint64_t)i, 0, ORC_P_INIT_POS, k, w);
            double r = s->R * sqrt(orc_uniform(w[0]));
            double th = 2.0 * ORC_PI * orc_uniform(w[1]);
            p[0] = r * cos(th);
            p[1] = r * sin(th);
            p[2] = s->H * (orc_uniform(w[2]) - 0.5);
            if (!orc_inside_grain(s, p)) { ok = 1; break; }
        }
        if (!ok) bad |= 1;
        uint64_t w[4];
        orc_draw(s, (uint64_t)i, 0, ORC_P_INIT_VEL, 0, w);
        double g1, g2, g3, g4;
        orc_box_muller(orc_uniform(w[0]), orc_uniform(w[1]), &g1, &g2);
        orc_box_muller(orc_uniform(w[2]), orc_uniform(w[3]), &g3, &g4);
        s->x[3 * i + 0] = p[0]; s->x[3 * i + 1] = p[1]; s->x[3 * i + 2] = p[2];
        s->v[3 * i + 0] = s->sig * g1;
        s->v[3 * i + 1] = s->sig * g2;
        if (s->flags & ORC_F_FIELD_DRIVEN) {
            /* time since the last collision: block (i, 0, INIT_VEL, 1), u0 */
            uint64_t w1[4];
            orc_draw(s, (uint64_t)i, 0, ORC_P_INIT_VEL, 1, w1);
            s->v[3 * i + 2] = s->sig * g3 - s->ufd * log(orc_uniform(w1[0]));
        } else {
            s->v[3 * i + 2] = s->u + s->sig * g3;
        }
    }
    for (int d = 0; d < s->nd; ++d) s->Q[d] = s->dq0[d];
    s->step = 0;
    s->nrec = 0;
    memset(s->sumQ, 0, sizeof s->sumQ);
    memset(s->sumF, 0, sizeof s->sumF);
    s->status = bad ? -4 : 0;
    return s->status;
}

/* ------------------------------------------------------------------------ */
/* Acceleration of ion i at the current positions and charges (Section 2):
 *   ion-ion: screened Coulomb (Yukawa, screening length r_De) field of every
 *            other superparticle of charge q;
 *   ion-dust: bare Coulomb field of each grain (asymmetric model);
 *   drive:   homogeneous field E along +z.
 * a_i = (e/mi) * E_total(x_i), the superparticle having the ion's q/m.     */
static void orc_accel_one(const orc_sys* s, int64_t i, double out[3])
{
    const double k = 1.0 / (4.0 * ORC_PI * ORC_EPS0);
    const double* xi = s->x + 3 * i;
    double ex = 0.0, ey = 0.0, ez = 0.0;
    if (!(s->flags & ORC_F_NO_ION_ION)) {
        for (int64_t j = 0; j < s->N; ++j) {
            if (j == i) continue;
            double dx = xi[0] - s->x[3 * j + 0];
            double dy = xi[1] - s->x[3 * j + 1];
            double dz = xi[2] - s->x[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double f;
            if (s->cut_on) {
                if (r >= s->r_cut) continue;
                /* switched energy phi(r) S(r): field -d(phi S)/dr along the unit vector */
                double phi = k * s->q * exp(-r / s->lam) / r;
                double dphi = -phi * (1.0 / r + 1.0 / s->lam);
                double S = 1.0, dS = 0.0;
                if (r > s->r_sw) {
                    double wd = s->r_cut - s->r_sw, x = (r - s->r_sw) / wd;
                    S = 1.0 - 6.0 * pow(x, 5) + 15.0 * pow(x, 4) - 10.0 * pow(x, 3);
                    dS = (-30.0 * pow(x, 4) + 60.0 * pow(x, 3) - 30.0 * pow(x, 2)) / wd;
                }
                f = -(dphi * S + phi * dS) / r;
            } else {
                f = k * s->q * (1.0 + r / s->lam) * exp(-r / s->lam) / (r * r * r);
            }
            ex += f * dx; ey += f * dy; ez += f * dz;
        }
    }
    for (int d = 0; d < s->nd; ++d) {
        double dx = xi[0] - s->dpos[d][0];
        double dy = xi[1] - s->dpos[d][1];
        double dz = xi[2] - s->dpos[d][2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double f = k * s->Q[d] / (r * r * r);
        ex += f * dx; ey += f * dy; ez += f * dz;
    }
    ez += s->E;
    if (s->conf_on) {
        double Eo[3];
        orc_confinement_field(s, xi, Eo);
        ex += Eo[0]; ey += Eo[1]; ez += Eo[2];
    }
    double qm = ORC_QE / s->mi;
    out[0] = qm * ex; out[1] = qm * ey; out[2] = qm * ez;
}

/* Accelerations of a subset of target ions (all ions as sources). */
void orc_accel_subset(const orc_sys* s, const int64_t* idx, int64_t n_idx, double* a)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_idx; ++t) orc_accel_one(s, idx[t], a + 3 * t);
}

/* Forces on the dust grains at the current state.
 *   Eq. (1): F_orbit,d = q Q_d/(4 pi eps0) sum_k (1 + rho/r_De) exp(-rho/r_De)
 *            (r_d - r_k)/rho^3 + Q_d E_out(r_d), the last term only while a
 *            confinement field is installed;
 *   Eq. (2): F_dd,d = Q_d/(4 pi eps0) sum_{p != d} Q_p (r_d - r_p)/|r_d - r_p|^3;
 *   Eq. (4): F_ext,d = Q_d E (along z).
 * Out: F[d][0] orbit, F[d][1] dust-dust, F[d][3] external (SI, N).        */
static void orc_dust_forces(const orc_sys* s, double F[][4][3])
{
    const double k = 1.0 / (4.0 * ORC_PI * ORC_EPS0);
    for (int d = 0; d < s->nd; ++d) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t i = 0; i < s->N; ++i) {
            double dx = s->dpos[d][0] - s->x[3 * i + 0];
            double dy = s->dpos[d][1] - s->x[3 * i + 1];
            double dz = s->dpos[d][2] - s->x[3 * i + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double f = (1.0 + r / s->lam) * exp(-r / s->lam) / (r * r * r);
            sx += f * dx; sy += f * dy; sz += f * dz;
        }
        double c = k * s->q * s->Q[d];
        F[d][0][0] = c * sx; F[d][0][1] = c * sy; F[d][0][2] = c * sz;
        if (s->conf_on) {
            double Eo[3];
            orc_confinement_field(s, s->dpos[d], Eo);
            for (int a = 0; a < 3; ++a) F[d][0][a] += s->Q[d] * Eo[a];
        }
        double px = 0.0, py = 0.0, pz = 0.0;
        for (int p = 0; p < s->nd; ++p) {
            if (p == d) continue;
            double dx = s->dpos[d][0] - s->dpos[p][0];
            double dy = s->dpos[d][1] - s->dpos[p][1];
            double dz = s->dpos[d][2] - s->dpos[p][2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double f = k * s->Q[d] * s->Q[p] / (r * r * r);
            px += f * dx; py += f * dy; pz += f * dz;
        }
        F[d][1][0] = px; F[d][1][1] = py; F[d][1][2] = pz;
        F[d][3][0] = 0.0; F[d][3][1] = 0.0; F[d][3][2] = s->Q[d] * s->E;
    }
}

/* Segment-sphere absorption test (Section 2: an ion intersecting the dust
 * surface during the step is removed).  Reading: the straight drift segment
 * x -> xh is tested, not only its end point.  Returns 1 and the entry
 * parameter t_hit in [0,1] if the segment comes within radius a of c.     */
static int orc_segment_hits(const double x[3], const double xh[3], const double c[3],
                            double a, double* t_hit)
{
    double sx = x[0] - c[0], sy = x[1] - c[1], sz = x[2] - c[2];
    double Dx = xh[0] - x[0], Dy = xh[1] - x[1], Dz = xh[2] - x[2];
    double DD = Dx * Dx + Dy * Dy + Dz * Dz;
    double sD = sx * Dx + sy * Dy + sz * Dz;
    double ss = sx * sx + sy * sy + sz * sz;
    double a2 = a * a;
    if (DD == 0.0) {
        if (ss <= a2) { *t_hit = 0.0; return 1; }
        return 0;
    }
    double t = -sD / DD;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double cx = sx + t * Dx, cy = sy + t * Dy, cz = sz + t * Dz;
    if (cx * cx + cy * cy + cz * cz > a2) return 0;
    double disc = sD * sD - DD * (ss - a2);
    if (disc < 0.0) disc = 0.0;
    double th = (-sD - sqrt(disc)) / DD;
    if (th < 0.0) th = 0.0;
    *t_hit = th;
    return 1;
}

/* Reinjection of one ion on the cylinder boundary (Appendix B).
 * Face: bottom if w0 < T_b, top if w0 < T_b + T_t, else side, with the
 * thresholds p * 2^64 of Eqs. (B.5)-(B.7).
 * Bottom (z = -H/2) / top (z = +H/2): position uniform on the disk,
 *   (x,y) = R sqrt(u1) (cos 2 pi u2, sin 2 pi u2); v_z from the flux-weighted
 *   distribution of Eq. (B.8) (bottom) or Eq. (B.9) (top, sign reversed);
 *   (v_x, v_y) Maxwellian, from the second block's (u0,u1).
 * Side: theta = 2 pi u1, z = H (u2 - 1/2); |v_r| = sig sqrt(-2 ln u3), the
 *   inverse of Eq. (B.12); v = -v_r r_hat (Eqs. B.10-B.11) + v_z z_hat with
 *   v_z ~ N(u, sig^2) from the second block's (u0,u1) (g1); unless the
 *   literal flag is set a tangential N(0, sig^2) part (g2) is added, which the
 *   product form of Eq. (B.1) implies.
 * Field-driven flow: phi(v_z) is the field-driven distribution above; the
 *   face fluxes and flux-weighted speeds use it, and a side ion takes
 *   v_z = sig g1 + ufd T with T = -ln u2 of the second block.              */
static void orc_reinject(const orc_sys* s, int64_t i, double x[3], double v[3])
{
    uint64_t b0[4], b1[4];
    orc_draw(s, (uint64_t)i, (uint64_t)s->step, ORC_P_REINJ, 0, b0);
    orc_draw(s, (uint64_t)i, (uint64_t)s->step, ORC_P_REINJ, 1, b1);
    double g1, g2;
    orc_box_muller(orc_uniform(b1[0]), orc_uniform(b1[1]), &g1, &g2);
    if (b0[0] < s->Tbt) {
        int bottom = b0[0] < s->Tb;
        double r = s->R * sqrt(orc_uniform(b0[1]));
        double th = 2.0 * ORC_PI * orc_uniform(b0[2]);
        x[0] = r * cos(th);
        x[1] = r * sin(th);
        x[2] = bottom ? -0.5 * s->H : 0.5 * s->H;
        v[0] = s->sig * g1;
        v[1] = s->sig * g2;
        if (s->flags & ORC_F_FIELD_DRIVEN)
            v[2] = bottom ? orc_fd_inverse(orc_uniform(b0[3]), s->ufd, s->sig, 0)
                          : -orc_fd_inverse(orc_uniform(b0[3]), s->ufd, s->sig, 1);
        else
            v[2] = bottom ? orc_flux_inverse(orc_uniform(b0[3]), s->u, s->sig)
                          : -orc_flux_inverse(orc_uniform(b0[3]), -s->u, s->sig);
    } else {
        double th = 2.0 * ORC_PI * orc_uniform(b0[1]);
        double c = cos(th), sn = sin(th);
        x[0] = s->R * c;
        x[1] = s->R * sn;
        x[2] = s->H * (orc_uniform(b0[2]) - 0.5);
        double vr = s->sig * sqrt(-2.0 * log(orc_uniform(b0[3])));
        double vt = (s->flags & ORC_F_LITERAL_SIDE) ? 0.0 : s->sig * g2;
        v[0] = -vr * c - vt * sn;
        v[1] = -vr * sn + vt * c;
        v[2] = (s->flags & ORC_F_FIELD_DRIVEN)
                   ? s->sig * g1 - s->ufd * log(orc_uniform(b1[2]))   /* phi(v_z), Eq. (B.1) */
                   : s->u + s->sig * g1;
    }
}

/* One time step n (Sections 2, Eqs. (1)-(4), Appendix B).
 *  1. forces on ions and dust at x^n, Q^n;
 *  2. kick v^ = v + dt a  (velocity Verlet in its staggered form: the
 *     stored velocity is the half-step one, one force evaluation per step);
 *  3. charge exchange at constant frequency: with probability
 *     P_c = 1 - exp(-nu dt) (decision w0 < T_c on block (i,n,COLL,0)) the
 *     velocity is replaced by a draw from the neutrals' Maxwellian at Ti
 *     (block (i,n,COLL,1): g1,g2 from (u0,u1), g3 from (u2,u3));
 *  4. drift x^ = x + dt v^;
 *  5. absorption: the segment x -> x^ meets a grain (smallest entry
 *     parameter wins, ties to the lower index); the grain counts the ion and
 *     collects its momentum m v^ (Eq. (3) with the superparticle mass);
 *  6. exit: x^2 + y^2 > R^2 or |z| > H/2 (equality is inside);
 *  7. charge: "given" keeps Q; "oml" adds (I_i^OML + I_e) dt; "consistent"
 *     adds q per absorbed superparticle plus I_e(Q^n) dt;
 *  8. F_coll = (sum of m v^)/dt, Eq. (3);
 *  9. absorbed and exited ions are reinjected (Appendix B);
 * 10. Q^n and the forces of step n are recorded; averages accumulate for
 *     n >= n_discard.                                                       */
int orc_step(orc_sys* s)
{
    const int64_t N = s->N;
    const double dt = s->dt;
    const int nd = s->nd;
    double F[ORC_MAXD][4][3];
    memset(F, 0, sizeof F);

    /* 1. */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) orc_accel_one(s, i, s->a + 3 * i);
    orc_dust_forces(s, F);

    double P[ORC_MAXD][3];
    int64_t cnt[ORC_MAXD];
    memset(P, 0, sizeof P);
    memset(cnt, 0, sizeof cnt);
    int64_t nexit = 0, ncoll = 0;
    double* xh = (double*)malloc((size_t)N * 3 * sizeof(double));
    double* vh = (double*)malloc((size_t)N * 3 * sizeof(double));
    if (!xh || !vh) { free(xh); free(vh); return -5; }

    /* 2-6, per ion. */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double* vi = vh + 3 * i;
        double* xi = xh + 3 * i;
        for (int c = 0; c < 3; ++c) vi[c] = s->v[3 * i + c] + dt * s->a[3 * i + c];
        s->hit[i] = 0;
        if (s->Pc > 0.0) {
            uint64_t w[4];
            orc_draw(s, (uint64_t)i, (uint64_t)s->step, ORC_P_COLL, 0, w);
            if (w[0] < s->Tc) {
                uint64_t b[4];
                double g1, g2, g3, g4;
                orc_draw(s, (uint64_t)i, (uint64_t)s->step, ORC_P_COLL, 1, b);
                orc_box_muller(orc_uniform(b[0]), orc_uniform(b[1]), &g1, &g2);
                orc_box_muller(orc_uniform(b[2]), orc_uniform(b[3]), &g3, &g4);
                vi[0] = s->sig * g1; vi[1] = s->sig * g2; vi[2] = s->sig * g3;
                s->hit[i] = 1;
            }
        }
        for (int c = 0; c < 3; ++c) xi[c] = s->x[3 * i + c] + dt * vi[c];
        int dhit = -1;
        double tbest = 2.0;
        for (int d = 0; d < nd; ++d) {
            double th;
            if (orc_segment_hits(s->x + 3 * i, xi, s->dpos[d], s->da[d], &th) && th < tbest) {
                tbest = th;
                dhit = d;
            }
        }
        if (dhit >= 0) {
            s->ev[i] = dhit;
        } else if (xi[0] * xi[0] + xi[1] * xi[1] > s->R * s->R || fabs(xi[2]) > 0.5 * s->H) {
            s->ev[i] = ORC_EV_EXITED;
        } else {
            s->ev[i] = ORC_EV_NONE;
        }
    }
    /* serial, index-ordered reductions of the per-ion events */
    for (int64_t i = 0; i < N; ++i) {
        ncoll += s->hit[i];
        if (s->ev[i] >= 0) {
            int d = s->ev[i];
            cnt[d] += 1;
            for (int c = 0; c < 3; ++c) P[d][c] += s->m * vh[3 * i + c];
        } else if (s->ev[i] == ORC_EV_EXITED) {
            nexit += 1;
        }
    }

    /* 7. */
    double Qn[ORC_MAXD];
    for (int d = 0; d < nd; ++d) Qn[d] = s->Q[d];
    for (int d = 0; d < nd; ++d) {
        if (s->mode == 1) {
            double Ii = orc_ion_current_oml(Qn[d], s->da[d], s->n, s->Ti, s->mi, s->u);
            double Ie = orc_electron_current(Qn[d], s->da[d], s->n, s->Te);
            s->Q[d] = Qn[d] + (Ii + Ie) * dt;
        } else if (s->mode == 2) {
            double Ie = orc_electron_current(Qn[d], s->da[d], s->n, s->Te);
            s->Q[d] = Qn[d] + s->q * (double)cnt[d] + Ie * dt;
        }
    }
    /* 8. */
    for (int d = 0; d < nd; ++d)
        for (int c = 0; c < 3; ++c) F[d][2][c] = P[d][c] / dt;

    /* 9. */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        if (s->ev[i] != ORC_EV_NONE) {
            orc_reinject(s, i, s->x + 3 * i, s->v + 3 * i);
        } else {
            for (int c = 0; c < 3; ++c) {
                s->x[3 * i + c] = xh[3 * i + c];
                s->v[3 * i + c] = vh[3 * i + c];
            }
        }
    }
    free(xh);
    free(vh);

    /* 10. */
    for (int d = 0; d < nd; ++d) {
        s->Qrec[d] = Qn[d];
        s->nabs[d] = cnt[d];
        for (int p = 0; p < 4; ++p)
            for (int c = 0; c < 3; ++c) s->F[d][p][c] = F[d][p][c];
    }
    s->nexit = nexit;
    s->ncoll = ncoll;
    if (s->step >= s->n_discard) {
        for (int d = 0; d < nd; ++d) {
            s->sumQ[d] += Qn[d];
            for (int p = 0; p < 4; ++p)
                for (int c = 0; c < 3; ++c) s->sumF[d][p][c] += F[d][p][c];
        }
        s->nrec += 1;
    }
    s->step += 1;
    for (int d = 0; d < nd; ++d)
        if (!isfinite(s->Q[d])) s->status = -3;
    return s->status;
}

int orc_run(orc_sys* s, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) {
        int st = orc_step(s);
        if (st) return st;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* State access (SI units: m, m/s, C). */
void orc_get_state(const orc_sys* s, double* x, double* v, double* Q, int64_t* step)
{
    if (x) memcpy(x, s->x, (size_t)s->N * 3 * sizeof(double));
    if (v) memcpy(v, s->v, (size_t)s->N * 3 * sizeof(double));
    if (Q) memcpy(Q, s->Q, (size_t)s->nd * sizeof(double));
    if (step) *step = s->step;
}

void orc_set_state(orc_sys* s, const double* x, const double* v, const double* Q, int64_t step)
{
    if (x) memcpy(s->x, x, (size_t)s->N * 3 * sizeof(double));
    if (v) memcpy(s->v, v, (size_t)s->N * 3 * sizeof(double));
    if (Q) memcpy(s->Q, Q, (size_t)s->nd * sizeof(double));
    s->step = step;
}

/* Outputs of the last step: accelerations [N][3], events [N], collision
 * flags [N], recorded charge [nd], forces [nd][4][3], absorbed counts [nd],
 * exit and collision totals. */
void orc_last_step(const orc_sys* s, double* a, int32_t* ev, int32_t* hit, double* Qrec,
                   double* F, int64_t* nabs, int64_t* nexit_ncoll)
{
    if (a) memcpy(a, s->a, (size_t)s->N * 3 * sizeof(double));
    if (ev) memcpy(ev, s->ev, (size_t)s->N * sizeof(int32_t));
    if (hit) memcpy(hit, s->hit, (size_t)s->N * sizeof(int32_t));
    if (Qrec) memcpy(Qrec, s->Qrec, (size_t)s->nd * sizeof(double));
    if (F) memcpy(F, s->F, (size_t)s->nd * 12 * sizeof(double));
    if (nabs) memcpy(nabs, s->nabs, (size_t)s->nd * sizeof(int64_t));
    if (nexit_ncoll) { nexit_ncoll[0] = s->nexit; nexit_ncoll[1] = s->ncoll; }
}

/* Time averages over the recorded steps: Q [nd], F [nd][4][3]; returns the
 * number of recorded steps. */
int64_t orc_averages(const orc_sys* s, double* Qavg, double* Favg)
{
    for (int d = 0; d < s->nd; ++d) {
        if (Qavg) Qavg[d] = s->nrec ? s->sumQ[d] / (double)s->nrec : 0.0;
        if (Favg)
            for (int p = 0; p < 4; ++p)
                for (int c = 0; c < 3; ++c)
                    Favg[12 * d + 3 * p + c] = s->nrec ? s->sumF[d][p][c] / (double)s->nrec : 0.0;
    }
    return s->nrec;
}

/* Dust forces of Eqs. (1), (2), (4) at the current state, without stepping. */
void orc_dust_forces_now(const orc_sys* s, double* F /*[nd][4][3]*/)
{
    double tmp[ORC_MAXD][4][3];
    memset(tmp, 0, sizeof tmp);
    orc_dust_forces(s, tmp);
    memcpy(F, tmp, (size_t)s->nd * 12 * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Confinement field of the outer plasma (Appendix A).
 *
 * Eqs. (A.1)-(A.2): the potential inside the cylindrical cavity is the
 * potential Phi0 of an infinite homogeneous ion background with Yukawa
 * screening, minus the screened Coulomb potential of the ions that fill the
 * cavity.  Reading: the ions of the sum are the superparticles at the time
 * of the call (the driver calls it once, right after orc_init); Phi0 is the
 * screened potential of the infinite background, n e r_De^2 / eps0 (that
 * is, k_B T_e / e).  Nodes r_k = k R / nx, z_p = p (H/2) / nz on the
 * half-plane y = 0, k = 0..nx, p = 0..nz; out[(nz+1) k + p] in volts.  An
 * ion exactly on a node is left out of that node's sum. */
void orc_confinement_grid(const orc_sys* s, int nx, int nz, double* out)
{
    const double k = 1.0 / (4.0 * ORC_PI * ORC_EPS0);
    const double phi0 = s->n * ORC_QE * s->lam * s->lam / ORC_EPS0;
    const int nn = (nx + 1) * (nz + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < nn; ++g) {
        const double gx = s->R * (double)(g / (nz + 1)) / (double)nx;
        const double gz = 0.5 * s->H * (double)(g % (nz + 1)) / (double)nz;
        double sum = 0.0;
        for (int64_t l = 0; l < s->N; ++l) {
            double dx = s->x[3 * l + 0] - gx;
            double dy = s->x[3 * l + 1];
            double dz = s->x[3 * l + 2] - gz;
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (d > 0.0) sum += exp(-d / s->lam) / d;
        }
        out[g] = phi0 - k * s->q * sum;
    }
}

/* Installs the fitted polynomial of Eq. (A.3), written in the scaled
 * variables (r/rs)^2 and (z/zs)^2: alpha[m] (volts) multiplies
 * (r/rs)^(2a_m) (z/zs)^(2b_m).  on = 0 removes the field. */
void orc_set_confinement(orc_sys* s, const double* alpha, double rs, double zs, int on)
{
    for (int m = 0; m < 15; ++m) s->conf_alpha[m] = alpha[m];
    s->conf_rs = rs;
    s->conf_zs = zs;
    s->conf_on = on ? 1 : 0;
}

/* Ion-ion cutoff (Section 4: a switching function that vanishes beyond a
 * fixed cutoff distance).  Reading: the screened Coulomb energy of a pair,
 * phi(r) = q^2 exp(-r/r_De) / (4 pi eps0 r), is multiplied by the smooth
 * step S(r) = 1 for r <= r_sw, 1 - 6x^5 + 15x^4 - 10x^3 with
 * x = (r - r_sw)/(r_cut - r_sw) between, 0 from r_cut on (the switching
 * function of the molecular-dynamics engine the paper runs on), and the
 * force is minus the gradient of phi S.  Only the ion-ion interaction is
 * switched; grain terms and the sum of Eq. (1) stay complete.  r_cut <= 0
 * restores the plain sum. */
void orc_set_cutoff(orc_sys* s, double r_sw, double r_cut)
{
    s->cut_on = r_cut > 0.0;
    s->r_sw = r_sw;
    s->r_cut = r_cut;
}

/* Exponents (powers of r and of z, as printed in Eq. (A.3)) of the terms. */
void orc_confinement_terms(int* r_pow, int* z_pow)
{
    for (int m = 0; m < 15; ++m) { r_pow[m] = 2 * ORC_PA[m]; z_pow[m] = 2 * ORC_PB[m]; }
}

/* P (volts) and E_out = -grad P (V/m) at n points x[n][3] (SI). */
void orc_confinement_eval(const orc_sys* s, int64_t n, const double* x, double* P, double* E)
{
    for (int64_t i = 0; i < n; ++i) {
        const double* xi = x + 3 * i;
        double u = (xi[0] * xi[0] + xi[1] * xi[1]) / (s->conf_rs * s->conf_rs);
        double v = xi[2] * xi[2] / (s->conf_zs * s->conf_zs);
        double p = 0.0;
        for (int m = 0; m < 15; ++m)
            p += s->conf_alpha[m] * orc_ipow(u, ORC_PA[m]) * orc_ipow(v, ORC_PB[m]);
        if (P) P[i] = p;
        if (E) orc_confinement_field(s, xi, E + 3 * i);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
