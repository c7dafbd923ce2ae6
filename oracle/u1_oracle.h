/*
 * u1_oracle.h -- plain FP64 CPU oracle for the compact U(1) multilevel hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This tree is the correctness reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or constant with the GPU library, and it never calls it.
 *
 * Everything here is written for readability: plain nested loops over sites,
 * plain complex products, plain left-to-right sums, in double precision,
 * compiled without floating-point contraction.  Each function names the part
 * of the paper (Amado, Cardoso, Bicudo, arXiv 1309.3859) it follows.
 *
 * Geometry (generic d in {2, 4}; time is the last axis, the paper's 0-hat):
 *   site  = x0 + L0*(x1 + L1*(x2 + L2*x3))
 *   link  = mu + d*site, mu = 0..d-1 (x, y, z, t in d = 4; x, t in d = 2)
 *   parity = (x0 + ... + x_{d-1}) mod 2, periodic wrap in every direction.
 */
#ifndef U1_ORACLE_H
#define U1_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox counter domains (fourth counter word). */
enum { ORC_DOM_HB = 0, ORC_DOM_INIT = 1, ORC_DOM_METRO = 2, ORC_DOM_TEST = 3 };

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the
 * published round description: out = bijection of ctr under key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Draw a von Mises(0, kappa) deviate by the Best--Fisher (1979) rejection
 * method, with random words taken from Philox blocks
 * (c0, c1, attempt_pair, domain) under key; see orc_vonmises in lattice.c.
 * Returns psi in [-pi, pi]; *n_attempts receives the number of attempts used
 * (-1 when the attempt cap is hit). */
double orc_vonmises(double kappa, const uint32_t key[2], uint32_t c0, uint32_t c1,
                    uint32_t domain, int* n_attempts);

void orc_vonmises_many(double kappa, uint32_t seed, uint32_t key_id, uint32_t c0_start, uint32_t c1,
                       uint32_t domain, long n, double* out, long* attempts_total);

typedef struct orc_lattice orc_lattice;

orc_lattice* orc_create(int d, const int* L, double beta, uint32_t seed, uint32_t key_id);
void orc_destroy(orc_lattice* lat);

/* start: 0 cold (all angles 0), 1 hot (uniform in [-pi, pi) from Philox). */
void orc_init(orc_lattice* lat, int start);

/* Canonical FP64 link view: th[mu + d*site]. */
void orc_get_links(const orc_lattice* lat, double* out);
void orc_set_links(orc_lattice* lat, const double* in);
uint32_t orc_get_counter(const orc_lattice* lat);
void orc_set_counter(orc_lattice* lat, uint32_t upd);

/* Staple sum A of link (site, mu): writes Re A, Im A. */
void orc_staple(const orc_lattice* lat, long site, int mu, double* are, double* aim);

/* Single-link updates (heatbath uses the lattice's current update counter). */
void orc_heatbath_link(orc_lattice* lat, long site, int mu);
void orc_overrelax_link(orc_lattice* lat, long site, int mu);
/* Metropolis with step delta (the lattice's current counter, domain METRO). */
void orc_metropolis_link(orc_lattice* lat, long site, int mu);
/* Stochastic update of sweeps: kind 0 heatbath (default), 2 Metropolis with
 * proposal step delta. */
void orc_set_update(orc_lattice* lat, int kind, double delta);

/* One checkerboard phase: all links of direction mu and the given parity that
 * are not frozen at slab thickness tau (tau <= 1: nothing frozen).
 * kind 0 = heatbath, 1 = overrelaxation, 2 = Metropolis.  Does not touch the
 * counter. */
void orc_phase(orc_lattice* lat, int kind, int mu, int parity, int tau);

/* One pass (8 phases in d = 4) and one sweep (stochastic pass, then n_or
 * overrelaxation passes).  A heatbath or Metropolis pass increments the
 * update counter. */
void orc_pass(orc_lattice* lat, int kind, int tau);
void orc_sweeps(orc_lattice* lat, int n, int n_or, int tau);

/* Plaquette angle theta_P of orientation (a, b) at site. */
double orc_plaq_angle(const orc_lattice* lat, long site, int a, int b);

/* Mean cos(theta_P) per absolute orientation, 6 slots:
 * E_x, E_y, E_z (P_{i t}), B_x (P_{yz}), B_y (P_{zx}), B_z (P_{xy}).
 * In d = 2 only slot 0 (P_{xt}) is filled. */
void orc_plaquette_means(const orc_lattice* lat, double out[6]);

/* Multilevel measurement specification. */
typedef struct {
    int n_levels;          /* 1 or 2 */
    int tau[2];            /* slab thickness, outer level first */
    int n_iter[2];         /* number of sublattice updates per level */
    int k_sweeps[2];       /* sweeps per sublattice update */
    int n_or;              /* overrelaxation passes per sweep */
    int n_dirs;            /* charge axes used in the sum over mu */
    int dirs[3];
    int n_r;
    const int* r;          /* separations */
    int n_probe;
    const int* probe;      /* n_probe x 4 ints: (l, p1, p2, mode) */
    int n_comp;
    const int* comp;       /* frame components 0..5 = E_par, E_perp1, E_perp2,
                              B_par, B_perp1, B_perp2 */
    int multihit;          /* 1: temporal links of the correlator averages [T]
                              replaced by their conditional means */
} orc_ml_spec;

/* I_1(kappa) / I_0(kappa) for kappa >= 0. */
double orc_bessel_ratio(double kappa);

/* Conditional mean of the link variable e^{i theta} of (site, mu) given
 * every other link: e^{-i arg A} I_1(beta |A|) / I_0(beta |A|) (0 if A = 0). */
void orc_link_mean(const orc_lattice* lat, long site, int mu, double* re, double* im);

/* Number of doubles one configuration's estimates occupy:
 * C[r] (re, im), CO[r][probe][comp][kind] (re, im), vacuum <O_sq>[6],
 * vacuum <O_lin>[6], binary exponent E[r].  kind 0 = O_sq, kind 1 = O_lin.
 * C and CO are mantissas: the estimate of separation r is the stored value
 * times 2^E[r] (products over slabs can leave the range of FP64). */
long orc_ml_result_size(const orc_ml_spec* spec);

/* One multilevel configuration (the body of the paper's Algorithm 1 with one
 * or two levels); writes orc_ml_result_size() doubles. Returns 0 on success. */
int orc_multilevel(orc_lattice* lat, const orc_ml_spec* spec, double* out);

/* Product of n complex factors (re[i], im[i]) as mantissa * 2^ex, rescaled
 * after every factor so that max(|re|, |im|) of the mantissa lies in [1, 2). */
void orc_scaled_product(long n, const double* re, const double* im, double* mre, double* mim, long* ex);

/* The final estimators of orc_multilevel from given slab averages:
 * at[((dir * n_r + r) * n_slabs + s) * n_sigma + x] and
 * ato[((((dir * n_r + r) * n_probe + p) * n_comp + c) * 2 + kind) * n_slabs + s) * n_sigma + x]
 * (complex, interleaved re, im); fills C, CO and E[r] of out (the vacuum
 * slots are left as they are).  Returns 0 on success. */
int orc_ml_finalize(const orc_ml_spec* spec, long n_sigma, int nt, int n_slabs, const double* at, const double* ato,
                    double* out);

#ifdef __cplusplus
}
#endif
#endif
