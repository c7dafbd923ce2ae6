/*
 * u1ml.h -- C ABI of libu1ml: the compact U(1) Luscher--Weisz multilevel hot
 * path on one AMD Instinct MI355X (gfx950).
 *
 * The calls follow the statement of the problem in Amado, Cardoso, Bicudo,
 * "Flux tube widening in compact U(1) lattice gauge theory computed at T < T_c
 * with the multilevel method and GPUs" (arXiv 1309.3859):
 *   - lattice Ns^3 x Nt with periodic boundaries, links U = exp(i theta),
 *     Wilson action with coupling beta                           (Sec. II)
 *   - sweeps of local link updates plus 3 overrelaxation steps    (Sec. II)
 *   - the multilevel hierarchy: time slabs of thickness tau whose boundary
 *     spatial links are frozen, n sublattice updates of k sweeps each, one
 *     or two levels                          (Sec. II.C, Algorithm 1)
 *   - Polyakov-loop correlators at separations r along a charge axis mu,
 *     and plaquette insertions (E and B components, O = 2 beta (1 - Re P)
 *     and sqrt(beta) Im P) at positions relative to the charge (Sec. II.C.3)
 *
 * Conventions
 *   - Nothing throws or aborts across this boundary; every call returns a
 *     u1ml_status.  One host thread per context at a time.
 *   - All pointers are owned by the caller except the context itself.  The
 *     device workspace is provided by the caller (for instance a torch uint8
 *     tensor) and is only borrowed by the context.
 *   - Calls marked "async" enqueue work on the context's stream and return;
 *     HIP errors they cause are reported by the next call that synchronises
 *     (U1ML_EDEVICE).
 *   - Results do not depend on the update kernel's tile shape, on how many
 *     ensembles share a launch, or on their order: every random number is a
 *     Philox4x32-10 block keyed by (seed, key_id) and countered by
 *     (link id, heatbath pass, attempt pair, domain), and every reduction runs
 *     in a fixed order with double-double partial sums.
 *   - Canonical link view (get/set): angle of link mu at site
 *     (x, y, z, t) is element mu + 4 * (x + Nx * (y + Ny * (z + Nz * t))),
 *     mu = 0, 1, 2, 3 = x, y, z, t.
 */
#ifndef U1ML_H
#define U1ML_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    U1ML_OK = 0,
    U1ML_EINVAL = 1,  /* invalid argument or problem description           */
    U1ML_ENOMEM = 2,  /* size overflow in the planner, or host allocation   */
    U1ML_EDEVICE = 3, /* a HIP call failed (message in u1ml_last_error)     */
    U1ML_ESTATE = 4,  /* call made in the wrong state (e.g. before init)    */
    U1ML_ENOTSUP = 5  /* not supported by the device or the runtime          */
} u1ml_status;

/* Errors common to every call: nothing throws or aborts across this
 * interface; every call returns a status and records a message for
 * u1ml_last_error.  EINVAL for a NULL context or output pointer, an
 * ensemble index outside [0, n_ens), a kind, direction, parity or count out
 * of range, a tau that is neither <= 1 nor one of the problem's level
 * thicknesses, or a host buffer of the wrong length.  ESTATE for updates,
 * timings, plaquettes or configurations before the links are set
 * (u1ml_init_links or u1ml_set_links), and for u1ml_multilevel with a full
 * results ring.  EDEVICE when a HIP call fails;
 * an asynchronous call's kernel errors surface at the next synchronising
 * call.  Calls on one context must come from one host thread at a time. */

enum { U1ML_FP64 = 0, U1ML_FP32 = 1 };         /* link storage / update arithmetic */
enum { U1ML_COLD = 0, U1ML_HOT = 1 };          /* start of u1ml_init_links         */
enum { U1ML_HEATBATH = 0, U1ML_OVERRELAX = 1, U1ML_METROPOLIS = 2 }; /* kind of u1ml_phase */

/* Stochastic update of every sweep (u1ml_problem.update); the paper uses
 * Metropolis (Sec. II).  Metropolis: one hit per link, proposal
 * theta' = theta + metro_delta (2 U1 - 1), accepted when U2 < exp(beta
 * (Re(e^{i theta'} A) - Re(e^{i theta} A))) with A the staple sum; U1, U2 from
 * the Philox block (link id, counter, 0, 2) of the ensemble's key. */
enum { U1ML_UPDATE_HEATBATH = 0, U1ML_UPDATE_METROPOLIS = 1 };

/* How the insertion estimators are contracted (Sec. II.C.3 defines what is
 * computed; both forms give the same estimator up to FP64 rounding):
 *   HISTORY:  per-site slab averages [TO](x) of every probe, formed from the
 *             stored measurements of the inner level; memory grows with the
 *             number of probes.
 *   SPECTRAL: the sum over sites of weight x T x O for every transverse
 *             displacement at once, by 2D discrete Fourier transforms over
 *             the plane orthogonal to the charge axis; with two levels the
 *             weights need the whole configuration's outer averages, so each
 *             configuration runs twice from the same start (the second pass
 *             replays the first bit for bit).  Memory does not grow with the
 *             number of probes.
 *   AUTO:     HISTORY unless its averages would exceed 16 GiB. */
enum { U1ML_FORM_AUTO = 0, U1ML_FORM_HISTORY = 1, U1ML_FORM_SPECTRAL = 2 };

/* One ensemble: Ns^3 x Nt lattice (Sec. II), coupling beta = 1/g^2 and its
 * Philox key.  Every extent must be even and >= 2 (checkerboard across the
 * periodic wrap); the index arithmetic of the kernels further needs
 * Nx Ny Nz / 2 < 2^24, Ny Nz < 2^22, Nt < 2^22 and the 4 V link words of
 * one ensemble below 4 GiB (V < 2^28 sites in FP32, 2^27 in FP64; e.g.
 * 256^3 x 14 in FP32), U1ML_EINVAL otherwise. */
typedef struct {
    int ns[3];
    int nt;
    double beta;
    uint32_t seed;
    uint32_t key_id;
} u1ml_ensemble;

/* One multilevel level (Algorithm 1): time slabs of thickness tau, with the
 * spatial links of the layers t = 0 mod tau frozen; n_iter sublattice updates
 * of k_sweeps sweeps each. */
typedef struct {
    int tau;
    int n_iter;
    int k_sweeps;
} u1ml_level;

/* Insertion position relative to the site x of the charge P^dagger(x), in the
 * charge frame (e_par = mu, e_perp1 = mu+1, e_perp2 = mu+2 mod 3):
 *   x0 = x + l_eff e_par + p1 e_perp1 + p2 e_perp2,
 *   l_eff = l                         if mode == 0,
 *   l_eff = l + l_mid(r, component)   if mode == 1 (mid-plane between the
 *           charges, Sec. III.B: floor((r-1)/2) for plaquettes spanning e_par,
 *           floor(r/2) otherwise). */
typedef struct {
    int l;
    int p1;
    int p2;
    int mode;
} u1ml_probe;

/* Problem description. Arrays are read during u1ml_plan / u1ml_create only.
 *   comps: frame components 0..5 = E_par, E_perp1, E_perp2 (plaquettes
 *          P_{i t}) and B_par, B_perp1, B_perp2 (P_{perp1 perp2},
 *          P_{perp2 par}, P_{par perp1}); for mu = x: E_x, E_y, E_z, B_x, B_y,
 *          B_z with B_x from P_{yz}, B_y from P_{zx}, B_z from P_{xy}.
 *   levels: outer first; with two levels the outer tau must be a multiple of
 *          the inner tau, and Nt a multiple of the outer tau.
 *   dirs:   charge axes (0, 1, 2) summed over in the estimators (Sec. II.C.3).
 *   max_configs: capacity of the device results ring (configurations).
 *   form:   U1ML_FORM_* (SPECTRAL needs every transverse plane of a charge
 *           axis to fit 64 KiB of complex doubles, i.e. at most 4096 sites;
 *           AUTO takes the form with the smaller estimated device time,
 *           u1ml_plan_info.est_history_ms / est_spectral_ms, from unit costs
 *           measured on MI355X, and the spectral form whenever the history
 *           form's per-site averages would exceed 64 GiB). */
typedef struct {
    int n_ens;
    const u1ml_ensemble* ens;
    int precision;
    int n_or;
    int n_levels;
    u1ml_level levels[2];
    int n_dirs;
    int dirs[3];
    int n_r;
    const int* r;
    int n_probe;
    const u1ml_probe* probes;
    int n_comp;
    const int* comps;
    int max_configs;
    int form;
    int update;          /* U1ML_UPDATE_* (0: heatbath)                      */
    double metro_delta;  /* Metropolis proposal step, 0 < delta <= pi         */
    int multihit;        /* 1: analytic multihit (Sec. II.C) of the temporal
                            links in the correlator averages [T]: each link
                            replaced by its conditional mean
                            e^{-i arg A} I_1(beta|A|)/I_0(beta|A|); at
                            separations whose temporal links share a
                            plaquette (r = 1 or Ns - 1) only the first end;
                            the insertion averages keep the plain links     */
    int ins_kernel;      /* history-form insertion contraction: 0 the kernel
                            estimated faster, 1 the vector kernel (FP64 FMA
                            per work-item), 2 the matrix-core kernel (FP64
                            MFMA steps; U1ML_ENOTSUP where its chunk does not
                            fit LDS); both compute the same sums            */
} u1ml_problem;

/* Planner output (bytes of each workspace section, 256-byte aligned). */
typedef struct {
    size_t ws_bytes;          /* total device workspace required             */
    size_t link_bytes;        /* link angles of every ensemble               */
    size_t history_bytes;     /* per-measurement slab phases and O sums      */
    size_t average_bytes;     /* slab averages [T], [TO] of the inner level  */
    size_t outer_bytes;       /* running sums of the outer level             */
    size_t result_bytes;      /* device results ring                         */
    size_t scratch_bytes;     /* reduction partials, tables, counters        */
    size_t paper_running_bytes; /* the paper's running-accumulator footprint
                                   2 * 8 * V * (area of the probe plane)/tau
                                   for comparison (Sec. II.D)                 */
    long n_doubles_per_config; /* doubles per ensemble per configuration:
                                  C[r] (re, im), CO[r][probe][comp][kind]
                                  (re, im), vacuum <O_sq>[6], <O_lin>[6],
                                  binary exponent E[r]; C and CO of
                                  separation r are mantissas, the estimate is
                                  the stored value times 2^E[r] (the products
                                  over slabs, Sec. II.C.2-3, can leave the
                                  range of FP64; E[r] is the largest exponent
                                  of the per-site correlator products)      */
    long updates_per_config;  /* non-frozen link updates of one multilevel
                                 configuration, all ensembles               */
    long updates_per_sweep;   /* link updates of one full-lattice sweep      */
    int form;                 /* the contraction form chosen (U1ML_FORM_HISTORY
                                 or U1ML_FORM_SPECTRAL)                       */
    size_t spectral_bytes;    /* weights, plane spectra, spectral sums and the
                                 replay copy of the links (SPECTRAL only)    */
    long launches_per_config; /* kernel launches of one u1ml_multilevel
                                 (upper bound)                              */
    double est_history_ms;    /* estimated device time per configuration that
                                 the insertion contraction adds in the history
                                 form (0 without probes)                    */
    double est_spectral_ms;   /* the same for the spectral form (-1 where it
                                 does not apply); AUTO takes the smaller     */
    int ins_slots;            /* history form: (probe, component) slots per
                                 block of the insertion contraction; 8 means
                                 the matrix-core kernel (16 x 16 x 4 FP64
                                 MFMA steps), 9, 6, 3 or 1 the vector kernel,
                                 whichever is estimated faster (0 without
                                 probes or in the spectral form)             */
} u1ml_plan_info;

typedef struct u1ml_ctx u1ml_ctx;

/* Pure host function: validates the problem (every rule returns U1ML_EINVAL
 * with a message for u1ml_last_error(NULL)) and sizes the workspace. */
u1ml_status u1ml_plan(const u1ml_problem* problem, u1ml_plan_info* out);

/* Creates a context on the current HIP device.  d_ws (device memory of at
 * least the planned ws_bytes, 256-byte aligned) and hip_stream (a hipStream_t,
 * may be NULL for the null stream) stay owned by the caller.  Uploads the
 * ensemble tables; links are undefined until u1ml_init_links. */
u1ml_status u1ml_create(const u1ml_problem* problem, void* d_ws, size_t ws_bytes, void* hip_stream,
                        u1ml_ctx** out);

/* Waits for the context's outstanding work on its stream, then frees host
 * state, graphs and the internal stream; never frees d_ws, which the caller
 * may release once this returns.  NULL is accepted.  The context is freed
 * even when the wait reports a device error (U1ML_EDEVICE). */
u1ml_status u1ml_destroy(u1ml_ctx* ctx);

/* Async.  Cold start (theta = 0) or hot start (theta = pi (2u - 1), u from
 * the Philox block (link, 0, 0, domain 1)); resets every update counter. */
u1ml_status u1ml_init_links(u1ml_ctx* ctx, int start);

/* Async.  n full-lattice sweeps (one heatbath pass, then n_or overrelaxation
 * passes; a pass visits mu = x, y, z, t, each even then odd sites) on every
 * ensemble (Sec. II). */
u1ml_status u1ml_sweeps(u1ml_ctx* ctx, int n);

/* Async.  One checkerboard phase (the even-then-odd update of Sec. II.D; the
 * local updates of Sec. II; the frozen boundary links of Sec. II.C.1 and
 * Algorithm 1): the links of direction mu and the given parity that are not
 * frozen at slab thickness tau (tau <= 1: none frozen), updated with kind
 * U1ML_HEATBATH, U1ML_OVERRELAX or U1ML_METROPOLIS (step metro_delta of the
 * problem), using the stochastic pass counter (device counter + pass_offset).
 * Does not advance the counter. */
u1ml_status u1ml_phase(u1ml_ctx* ctx, int kind, int mu, int parity, int tau, int pass_offset);

/* Async.  One multilevel configuration: the body of Algorithm 1 with the
 * problem's levels, then the slab products, appending one record of
 * n_doubles_per_config doubles per ensemble to the device results ring.
 * ESTATE when the ring is full or the links were never initialised. */
u1ml_status u1ml_multilevel(u1ml_ctx* ctx);

/* Synchronises.  Copies every record in the ring, configuration-major then
 * ensemble: host[(c * n_ens + e) * n_doubles_per_config + k]; *n_written is
 * the number of doubles copied (at most n_doubles).  Empties the ring. */
u1ml_status u1ml_copy_results(u1ml_ctx* ctx, double* host, size_t n_doubles, size_t* n_written);

/* Synchronise.  Canonical FP64 view of one ensemble's 4*V link angles. */
u1ml_status u1ml_get_links(u1ml_ctx* ctx, int ens, double* host, size_t n);
u1ml_status u1ml_set_links(u1ml_ctx* ctx, int ens, const double* host, size_t n);

/* Synchronise.  Heatbath pass counter of one ensemble (checkpoint / replay). */
u1ml_status u1ml_get_counter(u1ml_ctx* ctx, int ens, uint32_t* counter);
u1ml_status u1ml_set_counter(u1ml_ctx* ctx, int ens, uint32_t counter);

/* Synchronises.  Mean plaquette cos(theta_P) of the Wilson action (Sec. II;
 * the orientations of the field components of Sec. II.C.3) per ensemble and
 * absolute orientation (E_x, E_y, E_z from P_{i t}; B_x, B_y, B_z from P_{yz},
 * P_{zx}, P_{xy}): out[ens * 6 + o]. */
u1ml_status u1ml_plaquette(u1ml_ctx* ctx, double* out);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops): the plaquette means of
 * u1ml_plaquette, from the same kernels in the same order (bit-identical
 * values), enqueued on the context's stream and written to device memory
 * d_out[ens * 6 + o] (6 n_ens doubles, owned by the caller).  The
 * per-work-group partial sums go to a static device array of the library
 * (1.5 MiB on each GPU it runs on, held until the process ends) instead of
 * the workspace.  Allocates nothing and does not synchronise.  EINVAL for a
 * NULL d_out or more than 32 ensembles; ESTATE before the links are set.
 * Every call on a GPU shares that GPU's array and overwrites all the partial
 * sums it reads, so no call depends on what an earlier one left there; calls
 * that overlap in time on one GPU (other streams or contexts) race on the
 * array, and the caller must order them. */
u1ml_status u1ml_plaquette_noalloc(u1ml_ctx* ctx, double* d_out);

/* Synchronises.  Number of link angles that are not finite or lie outside
 * [-pi, pi] by more than 2^-20 relative, all ensembles. */
u1ml_status u1ml_health(u1ml_ctx* ctx, uint64_t* n_bad);

/* Times every candidate work-group size of the update kernels on this
 * problem (results are bit-identical for all of them) and keeps the fastest.
 * Synchronises; restores links and counters afterwards. */
typedef struct {
    int n_candidates;
    int block[8];
    double us_per_sweep[8];
    int chosen_block;
} u1ml_tune_report;
u1ml_status u1ml_autotune(u1ml_ctx* ctx, u1ml_tune_report* report);

/* Sets the update kernels' work-group size (64, 128, 256, 512 or 1024). */
u1ml_status u1ml_set_block(u1ml_ctx* ctx, int block);

/* Synchronises.  n_lanes = 2, 3 or 4 runs u1ml_sweeps and u1ml_multilevel
 * as that many lanes of about equal volume (ensembles dealt largest first) on
 * as many streams at once (the context's stream and internal ones, joined
 * back into the context's stream by events): a checkerboard phase lasts a
 * few microseconds, mostly launch and load latency, so phases of several
 * lanes side by side fill the device where one does not, and the
 * arithmetic-bound heatbath phases of one lane overlap the memory-bound
 * overrelaxation phases of another.  n_lanes = 1 runs the whole batch on the
 * context's stream.  Default: 2 lanes for FP32 links and 4 for FP64 links,
 * at most one per ensemble.  Every ensemble's
 * links and estimates are bit-identical for every lane count.  EINVAL for
 * n_lanes outside 1..4 or above the number of ensembles. */
u1ml_status u1ml_set_lanes(u1ml_ctx* ctx, int n_lanes);

/* 1: capture sweeps and multilevel bodies into HIP graphs (default);
 * 0: launch every kernel directly.  A multilevel body of more than 8192
 * kernel launches (u1ml_plan_info.launches_per_config) is always launched
 * directly. */
u1ml_status u1ml_set_graphs(u1ml_ctx* ctx, int enable);

/* Synchronises.  Average device time in microseconds of one launch of the
 * given checkerboard phase over the whole batch: n_rep launches on the
 * context's stream, each with a start/stop event pair that takes the
 * dispatch's own begin and end timestamps (hipExtLaunchKernelGGL), so launch
 * gaps are not counted.  These timestamps bracket the dispatch from its
 * processing to its completion signal, about 1 us more than the execution
 * window a kernel trace records for a launch of a few microseconds.  Links
 * change; counters do not. */
u1ml_status u1ml_time_phase(u1ml_ctx* ctx, int kind, int mu, int parity, int tau, int n_rep, double* us);

/* Synchronises.  u1ml_time_phase for one lane of the current split (lane
 * 0 .. n_lanes - 1; with one lane, the whole batch): that lane's launch of
 * the phase, as sweeps and configurations launch it, timed alone on the
 * context's stream; *bytes and *updates receive the lane's streaming-model
 * bytes and link updates of one launch (as u1ml_phase_bytes).  Links change;
 * counters do not.  EINVAL for a lane out of range. */
u1ml_status u1ml_time_phase_lane(u1ml_ctx* ctx, int lane, int kind, int mu, int parity, int tau, int n_rep,
                                 double* us, double* bytes, long* updates);

/* Algorithmic bytes moved by one launch of that phase under the streaming
 * model: every distinct link angle the phase reads once, every link it writes
 * once (heatbath 8 words per update, overrelaxation and Metropolis 9), all
 * ensembles. */
u1ml_status u1ml_phase_bytes(u1ml_ctx* ctx, int kind, int mu, int parity, int tau, double* bytes,
                             long* updates);

/* Async, no context.  Philox4x32-10 blocks on the device:
 * d_out[4 i + w] = word w of the block (c0 + i, c1, c2, c3) under key
 * (k0, k1), i < n.  d_out holds 4 n uint32. */
u1ml_status u1ml_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                             size_t n, uint32_t* d_out, void* hip_stream);

/* Async, no context.  n von Mises(0, kappa) draws with the heatbath's sampler
 * (Best--Fisher 1979) in the given precision; draw i uses Philox counter
 * words (c0 + i, c1) in domain 3 under key (seed, key_id).  d_out holds n
 * doubles; d_attempts (may be NULL) receives the attempt count per draw. */
u1ml_status u1ml_vonmises_fill(double kappa, int precision, uint32_t seed, uint32_t key_id, uint32_t c0,
                               uint32_t c1, size_t n, double* d_out, int* d_attempts, void* hip_stream);

/* Async, no context.  The library's FP64 sine and cosine (the staple sums of
 * Sec. II, the heatbath's envelope attempts, the slab phases and insertion
 * plaquettes of Sec. II.C) on n arguments with |x| < 2^22: d_s[i] = sin
 * d_x[i], d_c[i] = cos d_x[i], all three device arrays of n doubles owned by
 * the caller. */
u1ml_status u1ml_sincos_fill(const double* d_x, size_t n, double* d_s, double* d_c, void* hip_stream);

const char* u1ml_status_str(u1ml_status s);
/* Last error message of ctx, or of the last context-free call if ctx is NULL. */
const char* u1ml_last_error(const u1ml_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
