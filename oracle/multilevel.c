/*
 * multilevel.c -- oracle: the Luscher--Weisz multilevel estimators of the
 * Polyakov-loop correlator and of the plaquette (field) insertions.
 *
 * TEST INFRASTRUCTURE ONLY (see u1_oracle.h).  Plain FP64 complex arithmetic,
 * running accumulators per spatial site (the additional accumulator
 * lattices of Sec. II.D), plain left-to-right sums.
 *
 * Paper sections followed (arXiv 1309.3859):
 *  - two-link operator T(x,t,r) = U_0(x,t)^dagger U_0(x + r mu, t), and
 *    P^dagger(x) P(x + r mu) = prod_t T(x,t,r)                 (Sec. II.C.1)
 *  - slab operators: T^(2)(x,t,r) = T(x,t,r) T(x,t+1,r), averaged in slabs
 *    of thickness 2 with frozen boundaries; <P^dagger P> = < prod_s [T^(2)] >
 *                                                              (Sec. II.C.2)
 *  - two levels: T^(4) = [T^(2)(t)] [T^(2)(t+2)], Algorithm 1   (Sec. II.C.2)
 *  - field operators a^2 F = sqrt(beta) Im P, a^4 F^2 = 2 beta (1 - Re P);
 *    connected <O>_{P^dagger P} = <P^dagger P O>/<P^dagger P> - <O>;
 *    TO^(2) = [T^(2) (O(t) + O(t+1))],
 *    TO^(4) = [T^(2)(t)][TO^(2)(t+2)] + [TO^(2)(t)][T^(2)(t+2)],
 *    <P^dagger P O> = 1/(N_sigma N_t (d-1)) sum_x sum_mu sum_S [TO](S)
 *                     prod_{S' != S} [T](S')                   (Sec. II.C.3)
 * The slab thickness tau and the number of thin slabs per thick slab are
 * general here; the paper uses 2 and 2.
 */
#include "u1_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int orc__d(const orc_lattice* lat);
int orc__L(const orc_lattice* lat, int k);
long orc__V(const orc_lattice* lat);
double orc__beta(const orc_lattice* lat);
double orc__link(const orc_lattice* lat, long site, int mu);
long orc__shift(const orc_lattice* lat, long site, int mu, int n);

typedef struct {
    double re, im;
} cplx;

static cplx c_make(double re, double im)
{
    cplx z;
    z.re = re;
    z.im = im;
    return z;
}
static cplx c_mul(cplx a, cplx b) { return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static cplx c_conj(cplx a) { return c_make(a.re, -a.im); }
static cplx c_scale(cplx a, double s) { return c_make(a.re * s, a.im * s); }
static cplx c_phase(double th) { return c_make(cos(th), sin(th)); }

/* ---- charge frame ----------------------------------------------------------
 * For charge axis mu the frame is (e_par, e_perp1, e_perp2) = (mu, mu+1, mu+2)
 * mod 3.  Components 0..5 = E_par, E_perp1, E_perp2 (plaquettes P_{i t}) and
 * B_par, B_perp1, B_perp2 (P_{perp1 perp2}, P_{perp2 par}, P_{par perp1}),
 * so that for mu = x they are E_x, E_y, E_z, B_x, B_y, B_z with
 * B_x from P_{yz}, B_y from P_{zx}, B_z from P_{xy}. */
static void comp_plane(int d, int dir, int comp, int* a, int* b)
{
    int t = d - 1;
    int e0 = dir, e1 = (dir + 1) % 3, e2 = (dir + 2) % 3;
    if (d == 2) {
        *a = 0;
        *b = 1;
        return;
    }
    switch (comp) {
    case 0: *a = e0; *b = t; break;
    case 1: *a = e1; *b = t; break;
    case 2: *a = e2; *b = t; break;
    case 3: *a = e1; *b = e2; break;
    case 4: *a = e2; *b = e0; break;
    default: *a = e0; *b = e1; break;
    }
}

/* Mid-plane longitudinal offset (the paper evaluates profiles in the plane
 * half way between the charges, Sec. III.B; it is silent on odd r): a
 * plaquette spanning the charge axis sits at floor((r-1)/2), one orthogonal to
 * it at floor(r/2). */
static int l_mid(int r, int comp)
{
    int spans = (comp == 0 || comp == 4 || comp == 5);
    return spans ? (r - 1) / 2 : r / 2;
}

long orc_ml_result_size(const orc_ml_spec* sp)
{
    return 2L * sp->n_r + 4L * sp->n_r * sp->n_probe * sp->n_comp + 12L + sp->n_r;
}

typedef struct {
    const orc_lattice* lat;
    const orc_ml_spec* sp;
    int d, Nt;
    long V, Nsig;
    double beta, sqrt_beta;
} ctx_t;

static long idx_T(const ctx_t* c, int idir, int ir, int S, int s, long xs)
{
    return (((long)idir * c->sp->n_r + ir) * S + s) * c->Nsig + xs;
}

static long idx_TO(const ctx_t* c, int idir, int ir, int ip, int ic, int kind, int S, int s, long xs)
{
    long k = (((long)idir * c->sp->n_r + ir) * c->sp->n_probe + ip) * c->sp->n_comp + ic;
    k = k * 2 + kind;
    return (k * S + s) * c->Nsig + xs;
}

/* Spatial site of the insertion for charge site xs (spatial index, t = 0). */
static long probe_site(const ctx_t* c, long xs, int dir, int r, int ip, int comp)
{
    const int* pr = c->sp->probe + 4 * ip;
    int l = pr[0] + (pr[3] ? l_mid(r, comp) : 0);
    long y = orc__shift(c->lat, xs, dir, l);
    if (c->d == 4) {
        y = orc__shift(c->lat, y, (dir + 1) % 3, pr[1]);
        y = orc__shift(c->lat, y, (dir + 2) % 3, pr[2]);
    }
    return y;
}

/* One measurement inside the innermost level: adds the slab two-link products
 * T^(tau)(x, s, r) and T^(tau) * sum_{t in slab} O(x0, t) to the running sums,
 * and adds every plaquette's O to the vacuum sums. */
static void measure(const ctx_t* c, int tau, cplx* Tacc, cplx* TOacc, double* vsq, double* vlin)
{
    const orc_ml_spec* sp = c->sp;
    int S = c->Nt / tau;
    int tdir = c->d - 1;
    for (int idir = 0; idir < sp->n_dirs; ++idir) {
        int dir = sp->dirs[idir];
        for (int ir = 0; ir < sp->n_r; ++ir) {
            int r = sp->r[ir];
            for (long xs = 0; xs < c->Nsig; ++xs) {
                long xr = orc__shift(c->lat, xs, dir, r);
                /* multihit: both ends replaced by their conditional means,
                 * except when the two temporal links share a plaquette
                 * (neighbours: r = 1 or r = L - 1), then only the first */
                int adjacent = (r == 1 || r == orc__L(c->lat, dir) - 1);
                for (int s = 0; s < S; ++s) {
                    cplx T = c_make(1.0, 0.0), Tm = c_make(1.0, 0.0);
                    for (int t = s * tau; t < (s + 1) * tau; ++t) {
                        cplx u0 = c_phase(orc__link(c->lat, xs + c->Nsig * t, tdir));
                        cplx ur = c_phase(orc__link(c->lat, xr + c->Nsig * t, tdir));
                        T = c_mul(T, c_mul(c_conj(u0), ur));
                        if (sp->multihit) {
                            cplx m0, mr = ur;
                            orc_link_mean(c->lat, xs + c->Nsig * t, tdir, &m0.re, &m0.im);
                            if (!adjacent) orc_link_mean(c->lat, xr + c->Nsig * t, tdir, &mr.re, &mr.im);
                            Tm = c_mul(Tm, c_mul(c_conj(m0), mr));
                        }
                    }
                    long it = idx_T(c, idir, ir, S, s, xs);
                    /* [T] takes the multihit product; the insertions keep the
                     * plain links (their plaquettes can contain them) */
                    Tacc[it] = c_add(Tacc[it], sp->multihit ? Tm : T);
                    for (int ip = 0; ip < sp->n_probe; ++ip) {
                        for (int ic = 0; ic < sp->n_comp; ++ic) {
                            int comp = sp->comp[ic], a, b;
                            comp_plane(c->d, dir, comp, &a, &b);
                            long y = probe_site(c, xs, dir, r, ip, comp);
                            double osq = 0.0, olin = 0.0;
                            for (int t = s * tau; t < (s + 1) * tau; ++t) {
                                double thp = orc_plaq_angle(c->lat, y + c->Nsig * t, a, b);
                                osq += 2.0 * c->beta * (1.0 - cos(thp));
                                olin += c->sqrt_beta * sin(thp);
                            }
                            long i0 = idx_TO(c, idir, ir, ip, ic, 0, S, s, xs);
                            long i1 = idx_TO(c, idir, ir, ip, ic, 1, S, s, xs);
                            TOacc[i0] = c_add(TOacc[i0], c_scale(T, osq));
                            TOacc[i1] = c_add(TOacc[i1], c_scale(T, olin));
                        }
                    }
                }
            }
        }
    }
    /* vacuum <O>: every plaquette of every orientation */
    int n_orient = (c->d == 4) ? 6 : 1;
    for (int o = 0; o < n_orient; ++o) {
        int a, b;
        if (c->d == 2) {
            a = 0;
            b = 1;
        } else if (o < 3) {
            a = o;
            b = tdir;
        } else {
            a = (o == 3) ? 1 : (o == 4) ? 2 : 0;
            b = (o == 3) ? 2 : (o == 4) ? 0 : 1;
        }
        double ssq = 0.0, slin = 0.0;
        for (long site = 0; site < c->V; ++site) {
            double thp = orc_plaq_angle(c->lat, site, a, b);
            ssq += 2.0 * c->beta * (1.0 - cos(thp));
            slin += c->sqrt_beta * sin(thp);
        }
        vsq[o] += ssq;
        vlin[o] += slin;
    }
}

/* Products over slabs as a mantissa and a binary exponent.  The signal
 * <P^dagger P> falls exponentially with r N_t (about 1e-15 at the paper's
 * largest separations, Sec. II.C.2 and Fig. 4), and a lattice of many slabs
 * multiplies many averages of modulus below one, so a plain FP64 product can
 * leave the range of normal numbers.  After every factor the product is
 * rescaled by a power of two so that the larger of |re|, |im| lies in [1, 2);
 * a zero product stays zero. */
typedef struct {
    cplx m;
    long e;
} scplx;

static scplx s_norm(cplx m, long e)
{
    scplx z;
    double a = fmax(fabs(m.re), fabs(m.im));
    z.m = m;
    z.e = e;
    if (a == 0.0 || !isfinite(a)) return z;
    int k = ilogb(a);
    z.m = c_make(ldexp(m.re, -k), ldexp(m.im, -k));
    z.e = e + k;
    return z;
}

static scplx s_mul(scplx a, cplx b) { return s_norm(c_mul(a.m, b), a.e); }

static int s_zero(scplx a) { return a.m.re == 0.0 && a.m.im == 0.0; }

/* value of a * 2^-E as a plain double */
static cplx s_rel(scplx a, long E)
{
    long k = a.e - E;
    if (k < -2200) k = -2200; /* far below the smallest subnormal: zero */
    return c_make(ldexp(a.m.re, (int)k), ldexp(a.m.im, (int)k));
}

void orc_scaled_product(long n, const double* re, const double* im, double* mre, double* mim, long* ex)
{
    scplx p = s_norm(c_make(1.0, 0.0), 0);
    for (long i = 0; i < n; ++i) p = s_mul(p, c_make(re[i], im[i]));
    *mre = p.m.re;
    *mim = p.m.im;
    *ex = p.e;
}

/* Final estimators from slab averages AT[...][S][x] and ATO[...][S][x]:
 *   C(r)  = 1/(N_sigma |M|)     sum_mu sum_x prod_S [T](S)
 *   CO(r) = 1/(N_sigma |M| N_t) sum_mu sum_x sum_S [TO](S) prod_{S'!=S} [T](S')
 * written as mantissas relative to 2^E(r), E(r) the largest binary exponent
 * of the per-site products prod_S [T](S) (0 if all vanish), with E(r) stored
 * after the vacuum sums.  Two passes over the sites: the exponents first,
 * then the plain left-to-right sums of the rescaled terms. */
static void finalize(const orc_ml_spec* sp, long Nsig, int Nt, int S, const cplx* AT, const cplx* ATO, double* out)
{
    long base_co = 2L * sp->n_r;
    long base_e = 2L * sp->n_r + 4L * sp->n_r * sp->n_probe * sp->n_comp + 12L;
    double nC = 1.0 / ((double)Nsig * sp->n_dirs);
    double nCO = 1.0 / ((double)Nsig * sp->n_dirs * Nt);
    long n_items = (long)sp->n_dirs * Nsig;
    scplx* P = (scplx*)malloc(sizeof(scplx) * (size_t)(n_items > 0 ? n_items : 1));
    if (!P) return;
#define AT_(idir, ir, s, xs) AT[(((long)(idir) * sp->n_r + (ir)) * S + (s)) * Nsig + (xs)]
    for (int ir = 0; ir < sp->n_r; ++ir) {
        long E = 0;
        int any = 0;
        for (int idir = 0; idir < sp->n_dirs; ++idir) {
            for (long xs = 0; xs < Nsig; ++xs) {
                scplx p = s_norm(c_make(1.0, 0.0), 0);
                for (int s = 0; s < S; ++s) p = s_mul(p, AT_(idir, ir, s, xs));
                P[idir * Nsig + xs] = p;
                if (!s_zero(p) && (!any || p.e > E)) {
                    E = p.e;
                    any = 1;
                }
            }
        }
        cplx sumC = c_make(0.0, 0.0);
        for (long it = 0; it < n_items; ++it) sumC = c_add(sumC, s_rel(P[it], E));
        out[2 * ir + 0] = sumC.re * nC;
        out[2 * ir + 1] = sumC.im * nC;
        out[base_e + ir] = (double)E;
        for (int ip = 0; ip < sp->n_probe; ++ip) {
            for (int ic = 0; ic < sp->n_comp; ++ic) {
                for (int kind = 0; kind < 2; ++kind) {
                    long k = (((long)ir * sp->n_probe + ip) * sp->n_comp + ic) * 2 + kind;
                    cplx sumCO = c_make(0.0, 0.0);
                    for (int idir = 0; idir < sp->n_dirs; ++idir) {
                        for (long xs = 0; xs < Nsig; ++xs) {
                            for (int s = 0; s < S; ++s) {
                                long kk = ((long)idir * sp->n_r + ir) * sp->n_probe + ip;
                                kk = (kk * sp->n_comp + ic) * 2 + kind;
                                scplx term = s_norm(ATO[(kk * S + s) * Nsig + xs], 0);
                                for (int s2 = 0; s2 < S; ++s2) {
                                    if (s2 == s) continue;
                                    term = s_mul(term, AT_(idir, ir, s2, xs));
                                }
                                sumCO = c_add(sumCO, s_rel(term, E));
                            }
                        }
                    }
                    out[base_co + 2 * k + 0] = sumCO.re * nCO;
                    out[base_co + 2 * k + 1] = sumCO.im * nCO;
                }
            }
        }
    }
#undef AT_
    free(P);
}

int orc_ml_finalize(const orc_ml_spec* sp, long n_sigma, int nt, int n_slabs, const double* at, const double* ato,
                    double* out)
{
    if (n_sigma < 1 || nt < 1 || n_slabs < 1) return 1;
    finalize(sp, n_sigma, nt, n_slabs, (const cplx*)at, (const cplx*)ato, out);
    return 0;
}

static int check_spec(const orc_lattice* lat, const orc_ml_spec* sp)
{
    int d = orc__d(lat), Nt = orc__L(lat, d - 1);
    if (sp->n_levels < 1 || sp->n_levels > 2) return 1;
    for (int k = 0; k < sp->n_levels; ++k) {
        if (sp->tau[k] < 1 || Nt % sp->tau[k] != 0) return 2;
        if (sp->n_iter[k] < 1 || sp->k_sweeps[k] < 0) return 3;
    }
    if (sp->n_levels == 2 && sp->tau[0] % sp->tau[1] != 0) return 4;
    if (sp->n_dirs < 1 || sp->n_dirs > d - 1) return 5;
    for (int i = 0; i < sp->n_dirs; ++i)
        if (sp->dirs[i] < 0 || sp->dirs[i] >= d - 1) return 5;
    for (int i = 0; i < sp->n_comp; ++i) {
        if (sp->comp[i] < 0 || sp->comp[i] > 5) return 6;
        if (d == 2 && sp->comp[i] != 0) return 6;
    }
    return 0;
}

int orc_multilevel(orc_lattice* lat, const orc_ml_spec* sp, double* out)
{
    int err = check_spec(lat, sp);
    if (err) return err;
    ctx_t c;
    c.lat = lat;
    c.sp = sp;
    c.d = orc__d(lat);
    c.Nt = orc__L(lat, c.d - 1);
    c.V = orc__V(lat);
    c.Nsig = c.V / c.Nt;
    c.beta = orc__beta(lat);
    c.sqrt_beta = sqrt(c.beta);

    int two = (sp->n_levels == 2);
    int tau_i = two ? sp->tau[1] : sp->tau[0];
    int n_i = two ? sp->n_iter[1] : sp->n_iter[0];
    int k_i = two ? sp->k_sweeps[1] : sp->k_sweeps[0];
    int tau_o = sp->tau[0], n_o = two ? sp->n_iter[0] : 1, k_o = two ? sp->k_sweeps[0] : 0;
    int S_i = c.Nt / tau_i, S_o = c.Nt / tau_o, q = tau_o / tau_i;

    long nT_i = (long)sp->n_dirs * sp->n_r * S_i * c.Nsig;
    long nTO_i = nT_i * sp->n_probe * sp->n_comp * 2;
    long nT_o = (long)sp->n_dirs * sp->n_r * S_o * c.Nsig;
    long nTO_o = nT_o * sp->n_probe * sp->n_comp * 2;
    cplx* Tin = (cplx*)calloc((size_t)nT_i + 1, sizeof(cplx));
    cplx* TOin = (cplx*)calloc((size_t)nTO_i + 1, sizeof(cplx));
    cplx* Tout = two ? (cplx*)calloc((size_t)nT_o + 1, sizeof(cplx)) : NULL;
    cplx* TOout = two ? (cplx*)calloc((size_t)nTO_o + 1, sizeof(cplx)) : NULL;
    double vsq[6] = {0}, vlin[6] = {0};
    long n_meas = 0;
    if (!Tin || !TOin || (two && (!Tout || !TOout))) {
        free(Tin);
        free(TOin);
        free(Tout);
        free(TOout);
        return 10;
    }

    for (int ko = 0; ko < n_o; ++ko) {
        if (two) orc_sweeps(lat, k_o, sp->n_or, tau_o);
        memset(Tin, 0, sizeof(cplx) * (size_t)nT_i);
        memset(TOin, 0, sizeof(cplx) * (size_t)nTO_i);
        for (int m = 0; m < n_i; ++m) {
            orc_sweeps(lat, k_i, sp->n_or, tau_i);
            measure(&c, tau_i, Tin, TOin, vsq, vlin);
            n_meas++;
        }
        /* inner slab averages [T], [TO] */
        double inv_i = 1.0 / (double)n_i;
        for (long k = 0; k < nT_i; ++k) Tin[k] = c_scale(Tin[k], inv_i);
        for (long k = 0; k < nTO_i; ++k) TOin[k] = c_scale(TOin[k], inv_i);
        if (!two) break;
        /* combine q thin slabs into each thick slab (Sec. II.C.2-3) */
        for (int idir = 0; idir < sp->n_dirs; ++idir)
            for (int ir = 0; ir < sp->n_r; ++ir)
                for (long xs = 0; xs < c.Nsig; ++xs)
                    for (int S = 0; S < S_o; ++S) {
                        cplx T4 = c_make(1.0, 0.0);
                        for (int j = 0; j < q; ++j) T4 = c_mul(T4, Tin[idx_T(&c, idir, ir, S_i, S * q + j, xs)]);
                        long io = idx_T(&c, idir, ir, S_o, S, xs);
                        Tout[io] = c_add(Tout[io], T4);
                        for (int ip = 0; ip < sp->n_probe; ++ip)
                            for (int ic = 0; ic < sp->n_comp; ++ic)
                                for (int kind = 0; kind < 2; ++kind) {
                                    cplx TO4 = c_make(0.0, 0.0);
                                    for (int j = 0; j < q; ++j) {
                                        cplx term = TOin[idx_TO(&c, idir, ir, ip, ic, kind, S_i, S * q + j, xs)];
                                        for (int j2 = 0; j2 < q; ++j2) {
                                            if (j2 == j) continue;
                                            term = c_mul(term, Tin[idx_T(&c, idir, ir, S_i, S * q + j2, xs)]);
                                        }
                                        TO4 = c_add(TO4, term);
                                    }
                                    long k = idx_TO(&c, idir, ir, ip, ic, kind, S_o, S, xs);
                                    TOout[k] = c_add(TOout[k], TO4);
                                }
                    }
    }

    if (two) {
        double inv_o = 1.0 / (double)n_o;
        for (long k = 0; k < nT_o; ++k) Tout[k] = c_scale(Tout[k], inv_o);
        for (long k = 0; k < nTO_o; ++k) TOout[k] = c_scale(TOout[k], inv_o);
        finalize(sp, c.Nsig, c.Nt, S_o, Tout, TOout, out);
    } else {
        finalize(sp, c.Nsig, c.Nt, S_i, Tin, TOin, out);
    }
    long base_v = 2L * sp->n_r + 4L * sp->n_r * sp->n_probe * sp->n_comp;
    for (int o = 0; o < 6; ++o) {
        out[base_v + o] = vsq[o] / ((double)n_meas * (double)c.V);
        out[base_v + 6 + o] = vlin[o] / ((double)n_meas * (double)c.V);
    }
    free(Tin);
    free(TOin);
    free(Tout);
    free(TOout);
    return 0;
}
