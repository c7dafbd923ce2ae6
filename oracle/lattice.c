/*
 * lattice.c -- oracle: compact U(1) links, staples, heatbath, overrelaxation,
 * checkerboard phases with frozen time slabs, plaquettes.
 *
 * TEST INFRASTRUCTURE ONLY (see u1_oracle.h).  Plain FP64, plain loops.
 *
 * Paper: Amado, Cardoso, Bicudo, arXiv 1309.3859, Sec. II (lattice setup,
 * Wilson action with U = exp(i theta)), Sec. II.C.1 (sublattices between time
 * hyperplanes whose spatial links are held fixed), Algorithm 1 (nested update
 * loops), Sec. II.D (links stored as phases in double precision, even points
 * updated before odd points, in place).
 */
#include "u1_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.141592653589793
#define ORC_TWO_PI 6.283185307179586
#define ORC_MAX_ATTEMPTS 65536

struct orc_lattice {
    int d;
    int L[4];
    long V;
    double beta;
    uint32_t key[2];
    uint32_t upd;      /* stochastic pass counter (second Philox counter word) */
    int stoch;         /* stochastic update of a sweep: 0 heatbath, 2 Metropolis */
    double delta;      /* Metropolis step */
    long n_cap;        /* heatbath draws that hit the attempt cap */
    double* th;        /* th[mu + d*site] */
};

/* ---- geometry ---------------------------------------------------------- */

static void site_coords(const orc_lattice* lat, long site, int c[4])
{
    long s = site;
    for (int k = 0; k < 4; ++k) c[k] = 0;
    for (int k = 0; k < lat->d; ++k) {
        c[k] = (int)(s % lat->L[k]);
        s /= lat->L[k];
    }
}

static long coords_site(const orc_lattice* lat, const int c[4])
{
    long s = 0;
    for (int k = lat->d - 1; k >= 0; --k) s = s * lat->L[k] + c[k];
    return s;
}

/* Site displaced by n steps along direction mu, periodic. */
static long shift(const orc_lattice* lat, long site, int mu, int n)
{
    int c[4];
    site_coords(lat, site, c);
    int m = (c[mu] + n) % lat->L[mu];
    if (m < 0) m += lat->L[mu];
    c[mu] = m;
    return coords_site(lat, c);
}

static int parity_of(const orc_lattice* lat, long site)
{
    int c[4], s = 0;
    site_coords(lat, site, c);
    for (int k = 0; k < lat->d; ++k) s += c[k];
    return s & 1;
}

static double link(const orc_lattice* lat, long site, int mu)
{
    return lat->th[mu + (long)lat->d * site];
}

/* wrap(a) = a - 2 pi floor((a + pi) / (2 pi)), the representative in [-pi, pi). */
static double wrap(double a)
{
    return a - ORC_TWO_PI * floor((a + ORC_PI) / ORC_TWO_PI);
}

/* ---- create / init ------------------------------------------------------ */

orc_lattice* orc_create(int d, const int* L, double beta, uint32_t seed, uint32_t key_id)
{
    if (d != 2 && d != 4) return NULL;
    orc_lattice* lat = (orc_lattice*)calloc(1, sizeof(orc_lattice));
    if (!lat) return NULL;
    lat->d = d;
    lat->V = 1;
    for (int k = 0; k < 4; ++k) lat->L[k] = 1;
    for (int k = 0; k < d; ++k) {
        lat->L[k] = L[k];
        lat->V *= L[k];
    }
    lat->beta = beta;
    lat->key[0] = seed;
    lat->key[1] = key_id;
    lat->th = (double*)calloc((size_t)(lat->V * d), sizeof(double));
    if (!lat->th) {
        free(lat);
        return NULL;
    }
    return lat;
}

void orc_destroy(orc_lattice* lat)
{
    if (!lat) return;
    free(lat->th);
    free(lat);
}

/* Cold start: every U = 1.  Hot start: theta = pi (2u - 1) with u from word 0
 * of the Philox block (link, 0, 0, INIT), u = (w + 1/2) 2^-32. */
void orc_init(orc_lattice* lat, int start)
{
    long nl = lat->V * lat->d;
    for (long l = 0; l < nl; ++l) {
        if (start == 0) {
            lat->th[l] = 0.0;
        } else {
            uint32_t ctr[4] = {(uint32_t)l, 0u, 0u, ORC_DOM_INIT};
            uint32_t w[4];
            orc_philox4x32_10(ctr, lat->key, w);
            double u = ((double)w[0] + 0.5) * (1.0 / 4294967296.0);
            lat->th[l] = ORC_PI * (2.0 * u - 1.0);
        }
    }
    lat->upd = 0;
    lat->n_cap = 0;
}

void orc_get_links(const orc_lattice* lat, double* out)
{
    memcpy(out, lat->th, sizeof(double) * (size_t)(lat->V * lat->d));
}

void orc_set_links(orc_lattice* lat, const double* in)
{
    memcpy(lat->th, in, sizeof(double) * (size_t)(lat->V * lat->d));
}

uint32_t orc_get_counter(const orc_lattice* lat) { return lat->upd; }
void orc_set_counter(orc_lattice* lat, uint32_t upd) { lat->upd = upd; }

/* ---- staple (Sec. II, Wilson action) ------------------------------------
 * The action terms that contain theta_mu(x) are the plaquettes
 * P_{mu nu}(x) and P_{mu nu}(x - nu) for nu != mu.  Their angles are
 * theta_mu(x) + phi_f(nu) and theta_mu(x) + phi_b(nu) (the second up to an
 * overall sign, irrelevant for the cosine) with
 *   phi_f = th_nu(x+mu) - th_mu(x+nu) - th_nu(x)
 *   phi_b = th_nu(x-nu) - th_nu(x+mu-nu) - th_mu(x-nu).
 * A = sum_nu exp(i phi_f) + exp(i phi_b), nu ascending, forward first, so the
 * local action is -beta |A| cos(theta + arg A). */
void orc_staple(const orc_lattice* lat, long site, int mu, double* are, double* aim)
{
    double sr = 0.0, si = 0.0;
    long xp = shift(lat, site, mu, +1);
    for (int nu = 0; nu < lat->d; ++nu) {
        if (nu == mu) continue;
        long xpn = shift(lat, site, nu, +1);
        long xmn = shift(lat, site, nu, -1);
        long xpmn = shift(lat, xp, nu, -1);
        double phf = link(lat, xp, nu) - link(lat, xpn, mu) - link(lat, site, nu);
        double phb = link(lat, xmn, nu) - link(lat, xpmn, nu) - link(lat, xmn, mu);
        sr += cos(phf);
        si += sin(phf);
        sr += cos(phb);
        si += sin(phb);
    }
    *are = sr;
    *aim = si;
}

/* ---- von Mises sampler ---------------------------------------------------
 * Best, D. J. and Fisher, N. I. (1979), "Efficient simulation of the von
 * Mises distribution", Appl. Statist. 28, 152-157.  Envelope parameters:
 *   s = sqrt(1 + 4 kappa^2), tau = 1 + s,
 *   rho = (tau - sqrt(2 tau)) / (2 kappa), r = (1 + rho^2) / (2 rho);
 * rho is evaluated in the algebraically equal cancellation-free form
 *   rho = 2 kappa tau / ((s + 1) (tau + sqrt(2 tau))).
 * Attempt: z = cos(pi U1), f = (1 + r z) / (r + z), c = kappa (r - f);
 * accept if c (2 - c) - U2 > 0 or else if ln(c / U2) + 1 - c >= 0;
 * psi = sign * arccos(f).
 * Random words: attempt j uses the Philox block (c0, c1, j / 2, domain);
 * even j takes words (0, 1), odd j takes words (2, 3).  Of the pair (a, b):
 *   U1 = ((a >> 1) + 1/2) 2^-31, sign = -1 if (a & 1) else +1,
 *   U2 = (b + 1/2) 2^-32.
 * kappa = 0: psi = pi (2 U1 - 1) from attempt 0 (uniform). */
double orc_vonmises(double kappa, const uint32_t key[2], uint32_t c0, uint32_t c1,
                    uint32_t domain, int* n_attempts)
{
    uint32_t w[4];
    if (kappa == 0.0) {
        uint32_t ctr[4] = {c0, c1, 0u, domain};
        orc_philox4x32_10(ctr, key, w);
        double u1 = ((double)(w[0] >> 1) + 0.5) * (1.0 / 2147483648.0);
        if (n_attempts) *n_attempts = 1;
        return ORC_PI * (2.0 * u1 - 1.0);
    }
    double s = sqrt(1.0 + 4.0 * kappa * kappa);
    double tau = 1.0 + s;
    double rho = 2.0 * kappa * tau / ((s + 1.0) * (tau + sqrt(2.0 * tau)));
    double r = (1.0 + rho * rho) / (2.0 * rho);
    for (int j = 0; j < ORC_MAX_ATTEMPTS; ++j) {
        if ((j & 1) == 0) {
            uint32_t ctr[4] = {c0, c1, (uint32_t)(j >> 1), domain};
            orc_philox4x32_10(ctr, key, w);
        }
        uint32_t a = w[(j & 1) * 2 + 0];
        uint32_t b = w[(j & 1) * 2 + 1];
        double u1 = ((double)(a >> 1) + 0.5) * (1.0 / 2147483648.0);
        double sgn = (a & 1u) ? -1.0 : 1.0;
        double u2 = ((double)b + 0.5) * (1.0 / 4294967296.0);
        double z = cos(ORC_PI * u1);
        double f = (1.0 + r * z) / (r + z);
        if (f > 1.0) f = 1.0;
        if (f < -1.0) f = -1.0;
        double c = kappa * (r - f);
        int accept = (c * (2.0 - c) - u2 > 0.0);
        if (!accept) accept = (log(c / u2) + 1.0 - c >= 0.0);
        if (accept) {
            if (n_attempts) *n_attempts = j + 1;
            return sgn * acos(f);
        }
    }
    if (n_attempts) *n_attempts = -1;
    return 0.0;
}

/* ---- link updates --------------------------------------------------------
 * Heatbath: the conditional density of theta is proportional to
 * exp(beta |A| cos(theta + arg A)), so theta = psi - arg A with
 * psi ~ vonMises(0, beta |A|).  The paper uses Metropolis here (Sec. II);
 * the exact heatbath leaves the same local distribution invariant.
 * Overrelaxation (Sec. II, "3 steps of overrelaxation"): the reflection
 * theta -> -theta - 2 arg A keeps cos(theta + arg A), hence the action. */
void orc_heatbath_link(orc_lattice* lat, long site, int mu)
{
    double ar, ai;
    orc_staple(lat, site, mu, &ar, &ai);
    double R = sqrt(ar * ar + ai * ai);
    double phiA = atan2(ai, ar);
    uint32_t lid = (uint32_t)(mu + (long)lat->d * site);
    int na = 0;
    double psi = orc_vonmises(lat->beta * R, lat->key, lid, lat->upd, ORC_DOM_HB, &na);
    if (na < 0) {
        lat->n_cap++;
        return;
    }
    lat->th[mu + (long)lat->d * site] = wrap(psi - phiA);
}

/* Metropolis (the paper's update, Sec. II): propose theta' = theta + delta
 * (2 U1 - 1) and accept with probability min(1, exp(-dS)), where the local
 * action is -beta Re(e^{i theta} A) (the staple sum A collects every
 * plaquette containing the link), so
 *   -dS = beta [Re(e^{i theta'} A) - Re(e^{i theta} A)].
 * Random words: the Philox block (link id, counter, 0, ORC_DOM_METRO);
 * U1 = ((w0 >> 1) + 1/2) 2^-31 sets the proposal, U2 = (w1 + 1/2) 2^-32 the
 * decision: accept if -dS >= 0 or U2 < exp(-dS). */
void orc_metropolis_link(orc_lattice* lat, long site, int mu)
{
    double ar, ai;
    orc_staple(lat, site, mu, &ar, &ai);
    uint32_t lid = (uint32_t)(mu + (long)lat->d * site);
    uint32_t ctr[4] = {lid, lat->upd, 0u, ORC_DOM_METRO};
    uint32_t w[4];
    orc_philox4x32_10(ctr, lat->key, w);
    double u1 = ((double)(w[0] >> 1) + 0.5) * (1.0 / 2147483648.0);
    double u2 = ((double)w[1] + 0.5) * (1.0 / 4294967296.0);
    double th = lat->th[mu + (long)lat->d * site];
    double thn = wrap(th + lat->delta * (2.0 * u1 - 1.0));
    double dl = lat->beta * ((ar * cos(thn) - ai * sin(thn)) - (ar * cos(th) - ai * sin(th)));
    if (dl >= 0.0 || u2 < exp(dl)) lat->th[mu + (long)lat->d * site] = thn;
}

/* I_1(k)/I_0(k) from the ratio recurrence I_{n-1}/I_n = 2n/k + I_{n+1}/I_n,
 * i.e. the continued fraction 1/(2/k + 1/(4/k + 1/(6/k + ...))), evaluated
 * backwards from depth 40 + ceil(k) (relative error below 1e-15 for
 * k <= 100, checked against an independent Bessel implementation). */
double orc_bessel_ratio(double kappa)
{
    if (kappa <= 0.0) return 0.0;
    int depth = 40 + (int)ceil(kappa < 4000.0 ? kappa : 4000.0);
    double t = 0.0;
    for (int n = depth; n >= 1; --n) t = 1.0 / (2.0 * n / kappa + t);
    return t;
}

/* Analytic multihit (Sec. II.C; Parisi, Petronzio and Rapuano):
 * with every other link fixed, theta has density ~ exp(beta |A| cos(theta +
 * arg A)), so E[e^{i theta}] = e^{-i arg A} I_1(beta |A|) / I_0(beta |A|). */
void orc_link_mean(const orc_lattice* lat, long site, int mu, double* re, double* im)
{
    double ar, ai;
    orc_staple(lat, site, mu, &ar, &ai);
    double R = sqrt(ar * ar + ai * ai);
    if (R == 0.0) {
        *re = *im = 0.0;
        return;
    }
    double f = orc_bessel_ratio(lat->beta * R) / R;
    *re = ar * f;
    *im = -ai * f;
}

void orc_set_update(orc_lattice* lat, int kind, double delta)
{
    lat->stoch = kind;
    lat->delta = delta;
}

void orc_overrelax_link(orc_lattice* lat, long site, int mu)
{
    double ar, ai;
    orc_staple(lat, site, mu, &ar, &ai);
    if (ar == 0.0 && ai == 0.0) return;
    double phiA = atan2(ai, ar);
    double th = lat->th[mu + (long)lat->d * site];
    lat->th[mu + (long)lat->d * site] = wrap(-th - 2.0 * phiA);
}

/* ---- checkerboard phases and frozen slabs --------------------------------
 * Links of one direction and one parity share no plaquette, so they can be
 * updated at once and in place (Sec. II.D: even points, then odd points).
 * Sublattice updates (Sec. II.C.1, Algorithm 1) keep the spatial links of the
 * time layers t = 0 mod tau fixed; temporal links are always updated. */
static int frozen(const orc_lattice* lat, long site, int mu, int tau)
{
    if (tau <= 1 || mu == lat->d - 1) return 0;
    int c[4];
    site_coords(lat, site, c);
    return (c[lat->d - 1] % tau) == 0;
}

void orc_phase(orc_lattice* lat, int kind, int mu, int parity, int tau)
{
    for (long site = 0; site < lat->V; ++site) {
        if (parity_of(lat, site) != parity) continue;
        if (frozen(lat, site, mu, tau)) continue;
        if (kind == 0)
            orc_heatbath_link(lat, site, mu);
        else if (kind == 2)
            orc_metropolis_link(lat, site, mu);
        else
            orc_overrelax_link(lat, site, mu);
    }
}

/* One pass: directions x, y, z, t in turn, each even parity then odd. */
void orc_pass(orc_lattice* lat, int kind, int tau)
{
    for (int mu = 0; mu < lat->d; ++mu)
        for (int p = 0; p < 2; ++p) orc_phase(lat, kind, mu, p, tau);
    if (kind == 0 || kind == 2) lat->upd++;
}

/* One sweep: a stochastic pass (heatbath, or Metropolis after
 * orc_set_update) followed by n_or overrelaxation passes. */
void orc_sweeps(orc_lattice* lat, int n, int n_or, int tau)
{
    for (int i = 0; i < n; ++i) {
        orc_pass(lat, lat->stoch, tau);
        for (int k = 0; k < n_or; ++k) orc_pass(lat, 1, tau);
    }
}

/* ---- plaquettes (Sec. II) ------------------------------------------------
 * P_{ab}(y) = U_a(y) U_b(y+a) U_a(y+b)^-1 U_b(y)^-1. */
double orc_plaq_angle(const orc_lattice* lat, long site, int a, int b)
{
    long ya = shift(lat, site, a, +1);
    long yb = shift(lat, site, b, +1);
    return link(lat, site, a) + link(lat, ya, b) - link(lat, yb, a) - link(lat, site, b);
}

void orc_plaquette_means(const orc_lattice* lat, double out[6])
{
    static const int planes4[6][2] = {{0, 3}, {1, 3}, {2, 3}, {1, 2}, {2, 0}, {0, 1}};
    for (int o = 0; o < 6; ++o) out[o] = 0.0;
    int n_orient = (lat->d == 4) ? 6 : 1;
    for (int o = 0; o < n_orient; ++o) {
        int a = (lat->d == 4) ? planes4[o][0] : 0;
        int b = (lat->d == 4) ? planes4[o][1] : 1;
        double s = 0.0;
        for (long site = 0; site < lat->V; ++site) s += cos(orc_plaq_angle(lat, site, a, b));
        out[o] = s / (double)lat->V;
    }
}

/* Accessors used by multilevel.c. */
int orc__d(const orc_lattice* lat) { return lat->d; }
int orc__L(const orc_lattice* lat, int k) { return lat->L[k]; }
long orc__V(const orc_lattice* lat) { return lat->V; }
double orc__beta(const orc_lattice* lat) { return lat->beta; }
double orc__link(const orc_lattice* lat, long site, int mu) { return link(lat, site, mu); }
long orc__shift(const orc_lattice* lat, long site, int mu, int n) { return shift(lat, site, mu, n); }
long orc__n_cap(const orc_lattice* lat) { return lat->n_cap; }

/* Many independent von Mises draws for the sampler tests: draw i uses the
 * Philox counter words (c0_start + i, c1) in the given domain. */
void orc_vonmises_many(double kappa, uint32_t seed, uint32_t key_id, uint32_t c0_start, uint32_t c1,
                       uint32_t domain, long n, double* out, long* attempts_total)
{
    uint32_t key[2] = {seed, key_id};
    long tot = 0;
    for (long i = 0; i < n; ++i) {
        int na = 0;
        out[i] = orc_vonmises(kappa, key, c0_start + (uint32_t)i, c1, domain, &na);
        tot += na;
    }
    if (attempts_total) *attempts_total = tot;
}
