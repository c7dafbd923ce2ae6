// u1ml_api.cpp -- host side of libu1ml: planner, workspace layout, the
// Algorithm-1 scheduler (Amado, Cardoso, Bicudo, arXiv 1309.3859, Sec. II.C)
// with HIP-graph capture, and the C ABI declared in include/u1ml.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/u1ml.h"
#include "u1ml_internal.hpp"

using namespace u1ml;

namespace {

thread_local std::string g_err;  // context-free error text

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool mul_ok(size_t a, size_t b, size_t* out) { return !__builtin_mul_overflow(a, b, out); }
bool add_ok(size_t a, size_t b, size_t* out) { return !__builtin_add_overflow(a, b, out); }

struct Sizes {
    // per ensemble element offsets
    std::vector<size_t> links, hc, ho, at, ato, ot, oto, vac;
    std::vector<size_t> wf, gf, sph, spo, facc;  // spectral form (double2 elements)
    std::vector<size_t> cpl, opl;                // plane-major copies (double2, real elements)
};

struct Layout {
    size_t off_links, off_hc, off_ho, off_at, off_ato, off_ot, off_oto, off_res, off_scr;
    size_t sz_links, sz_hc, sz_ho, sz_at, sz_ato, sz_ot, sz_oto, sz_res, sz_scr;
    // spectral form: weights W, G; plane spectra of T and O; spectral sums; replay copy of the links
    size_t off_wf, off_gf, off_sph, off_spo, off_facc, off_saved, off_cpl, off_opl;
    size_t sz_wf, sz_gf, sz_sph, sz_spo, sz_facc, sz_saved, sz_cpl, sz_opl;
    // scratch sub-offsets (bytes from off_scr)
    size_t s_ens, s_obs, s_r, s_probe, s_comp, s_bstart, s_upd, s_ring, s_vpart, s_ppart, s_pout, s_count,
        s_stage, s_bmap, s_mmap, s_prodpart, s_pgroup, s_gdesc, s_pblk;
    // the lanes' descriptors and tables (each sized for the whole batch)
    size_t s_lens[4], s_lbstart[4], s_lbmap[4], s_lmmap[4], s_lring[4];
    size_t bmap_stride;  // entries per update class (blocks of 64 threads)
    int n_bstart_tables;
};

constexpr int kTabUpd = 0;    // 4 update classes
constexpr int kTabAll = 4;    // all links (init, health)
constexpr int kTabMeas = 5;   // spatial sites
constexpr int kTabCon = 6;    // contraction items
constexpr int kTabComb = 7;   // combine items
constexpr int kTabProd = 8;   // slab-product work-groups
constexpr int kTabSite = 9;   // spectral weights: (axis, r, site) items
constexpr int kTabPlane = 10; // spectral plane transforms: work-groups
constexpr int kTabMac = 11;   // spectral sums: work-groups
constexpr int kTabStage = 12; // spectral staging: work-groups
constexpr int kTabIns = 13;   // insertion contraction: work-groups
constexpr int kNumTabs = 14;
constexpr int kXcds = 8;  // accelerator complex dies of an MI355X, each with its own L2
constexpr int kMaxLanes = 4;  // streams that sweeps and configurations are spread over
// lanes a context starts with: FP32 phases are short enough that two lanes
// fill the device and a third adds under 1 %; the longer, arithmetic-bound
// FP64 phases gain about 2.5 % more from four (C4 on MI355X: FP32 8.50,
// 8.43, 8.64 ms per configuration with 2, 3, 4 lanes; FP64 17.96, 17.78, 17.56)
int default_lanes(int precision) { return precision == U1ML_FP64 ? 4 : 2; }

struct Problem {
    int n_ens = 0;
    std::vector<u1ml_ensemble> ens;
    int precision = 0, n_or = 3, n_levels = 1;
    u1ml_level lv[2] = {};
    int n_dirs = 1;
    int dirs[3] = {0, 0, 0};
    std::vector<int> r;
    std::vector<u1ml_probe> probes;
    std::vector<int> comps;
    int max_configs = 1;
    int form_req = U1ML_FORM_AUTO;
    int update = U1ML_UPDATE_HEATBATH;
    bool multihit = false;
    int ins_kernel = 0;  // 0: estimated faster, 1: vector, 2: matrix cores
    double metro_delta = 1.0;
    // derived
    int tau_i = 2, n_i = 1, k_i = 1, tau_o = 2, n_o = 1, k_o = 0;
    bool two = false;
    bool spectral = false;        // insertion contraction in the spectral form
    double est_hist_ms = 0.0, est_spec_ms = -1.0;  // the planner's cost estimates of the two forms
    std::vector<int> pgroup;      // probe -> group of probes sharing (l, mode)
    std::vector<int> gdesc;       // group -> (l, mode)
    std::vector<int> pblk;        // insertion contraction: slot blocks, kInsBlkInts ints each
    int ins_ks = 1;               // insertion contraction: slots per block (kMfSlots: matrix cores)
    // insertion slot keys: (l, mode, spans) and their (probe, component index) slots
    std::vector<std::vector<std::pair<int, int>>> skeys;
    std::vector<int> skey_l, skey_mode, skey_spans;
    int ins_ks_vec = 1;           // the vector kernel's slots per block
    bool ins_mfma_est = false;    // the matrix-core kernel is estimated faster (and applies)
    long long nd_cfg = 0;
};

// frame components whose plaquette spans the charge axis: E_par (P_{par t}),
// B_perp1 (P_{perp2 par}) and B_perp2 (P_{par perp1})
bool comp_spans_axis_host(int c) { return c == 0 || c == 4 || c == 5; }

bool fail(std::string* err, const std::string& msg)
{
    if (err) *err = msg;
    return false;
}

// slot blocks of ks slots (kInsBlkInts ints each): l, mode, spans, number of
// slots, then per slot probe, component index, p1, p2
void pack_slot_blocks(Problem* P, int ks)
{
    P->pblk.clear();
    P->ins_ks = ks;
    for (size_t kk = 0; kk < P->skeys.size(); ++kk) {
        const auto& key = P->skeys[kk];
        for (size_t b = 0; b < key.size(); b += ks) {
            int blk[kInsBlkInts] = {};
            blk[0] = P->skey_l[kk];
            blk[1] = P->skey_mode[kk];
            blk[2] = P->skey_spans[kk];
            blk[3] = (int)std::min<size_t>(ks, key.size() - b);
            for (int k = 0; k < blk[3]; ++k) {
                const int p = key[b + k].first, ic = key[b + k].second;
                blk[4 + 4 * k] = p;
                blk[5 + 4 * k] = ic;
                blk[6 + 4 * k] = P->probes[p].p1;
                blk[7 + 4 * k] = P->probes[p].p2;
            }
            P->pblk.insert(P->pblk.end(), blk, blk + kInsBlkInts);
        }
    }
}

bool read_problem(const u1ml_problem* p, Problem* P, std::string* err)
{
    if (!p) return fail(err, "problem is NULL");
    if (p->n_ens < 1 || !p->ens) return fail(err, "n_ens must be >= 1 with a non-NULL ensemble array");
    if (p->precision != U1ML_FP64 && p->precision != U1ML_FP32) return fail(err, "precision must be 0 (FP64) or 1 (FP32)");
    if (p->n_or < 0) return fail(err, "n_or must be >= 0");
    if (p->update != U1ML_UPDATE_HEATBATH && p->update != U1ML_UPDATE_METROPOLIS)
        return fail(err, "update must be 0 (heatbath) or 1 (Metropolis)");
    if (p->update == U1ML_UPDATE_METROPOLIS && !(p->metro_delta > 0.0 && p->metro_delta <= M_PI))
        return fail(err, "metro_delta must satisfy 0 < delta <= pi");
    P->update = p->update;
    if (p->multihit != 0 && p->multihit != 1) return fail(err, "multihit must be 0 or 1");
    P->multihit = p->multihit == 1;
    if (p->ins_kernel < 0 || p->ins_kernel > 2) return fail(err, "ins_kernel must be 0, 1 or 2");
    P->ins_kernel = p->ins_kernel;
    P->metro_delta = p->metro_delta;
    if (p->n_levels < 1 || p->n_levels > 2) return fail(err, "n_levels must be 1 or 2");
    if (p->max_configs < 1) return fail(err, "max_configs must be >= 1");
    P->n_ens = p->n_ens;
    P->ens.assign(p->ens, p->ens + p->n_ens);
    P->precision = p->precision;
    P->n_or = p->n_or;
    P->n_levels = p->n_levels;
    P->lv[0] = p->levels[0];
    P->lv[1] = p->levels[1];
    P->max_configs = p->max_configs;
    for (int k = 0; k < p->n_levels; ++k) {
        const u1ml_level& L = p->levels[k];
        if (L.tau < 2) return fail(err, "level tau must be >= 2 (a slab needs a frozen boundary layer)");
        if (L.n_iter < 1) return fail(err, "level n_iter must be >= 1");
        if (L.k_sweeps < 0) return fail(err, "level k_sweeps must be >= 0");
    }
    P->two = (p->n_levels == 2);
    if (P->two) {
        P->tau_o = p->levels[0].tau;
        P->n_o = p->levels[0].n_iter;
        P->k_o = p->levels[0].k_sweeps;
        P->tau_i = p->levels[1].tau;
        P->n_i = p->levels[1].n_iter;
        P->k_i = p->levels[1].k_sweeps;
        if (P->tau_o % P->tau_i != 0) return fail(err, "outer tau must be a multiple of the inner tau");
        if (P->tau_o / P->tau_i > 8) return fail(err, "at most 8 inner slabs per outer slab");
    } else {
        P->tau_i = P->tau_o = p->levels[0].tau;
        P->n_i = p->levels[0].n_iter;
        P->k_i = p->levels[0].k_sweeps;
        P->n_o = 1;
        P->k_o = 0;
    }
    if (p->n_dirs < 1 || p->n_dirs > 3) return fail(err, "n_dirs must be 1..3");
    P->n_dirs = p->n_dirs;
    for (int i = 0; i < p->n_dirs; ++i) {
        if (p->dirs[i] < 0 || p->dirs[i] > 2) return fail(err, "charge axes must be 0, 1 or 2");
        for (int j = 0; j < i; ++j)
            if (p->dirs[j] == p->dirs[i]) return fail(err, "charge axes must be distinct");
        P->dirs[i] = p->dirs[i];
    }
    if (p->n_r < 1 || !p->r) return fail(err, "n_r must be >= 1 with a non-NULL r array");
    P->r.assign(p->r, p->r + p->n_r);
    if (p->n_probe < 0 || (p->n_probe > 0 && !p->probes)) return fail(err, "bad probe array");
    if (p->n_probe > 0) P->probes.assign(p->probes, p->probes + p->n_probe);
    if (p->n_comp < 0 || p->n_comp > 6 || (p->n_comp > 0 && !p->comps)) return fail(err, "n_comp must be 0..6");
    if (p->n_comp > 0) P->comps.assign(p->comps, p->comps + p->n_comp);
    for (int c : P->comps)
        if (c < 0 || c > 5) return fail(err, "components must be 0..5");
    if (P->probes.empty() != P->comps.empty()) return fail(err, "probes and components must both be given or both be empty");
    for (int e = 0; e < P->n_ens; ++e) {
        const u1ml_ensemble& E = P->ens[e];
        const int ext[4] = {E.ns[0], E.ns[1], E.ns[2], E.nt};
        for (int k = 0; k < 4; ++k)
            if (ext[k] < 2 || ext[k] % 2 != 0) return fail(err, "every extent must be even and >= 2 (ensemble " + std::to_string(e) + ")");
        if (!std::isfinite(E.beta) || E.beta < 0) return fail(err, "beta must be finite and >= 0");
        if (E.nt % P->tau_o != 0) return fail(err, "Nt must be a multiple of the outer tau");
        if (E.nt % P->tau_i != 0) return fail(err, "Nt must be a multiple of the inner tau");
        const double V = (double)E.ns[0] * E.ns[1] * E.ns[2] * E.nt;
        if (4.0 * V >= 4294967296.0) return fail(err, "4 V must fit in 32 bits (link ids)");
        // the kernels address an ensemble's links with 32-bit byte offsets
        if (4.0 * V * (P->precision == U1ML_FP64 ? 8 : 4) >= 4294967296.0)
            return fail(err, "the links of one ensemble (4 V words) must stay below 4 GiB");
        if ((double)E.ns[1] * E.ns[2] >= 4194304.0) return fail(err, "Ny * Nz must be below 2^22");
        if (E.nt >= 4194304) return fail(err, "Nt must be below 2^22");
        if ((double)E.ns[0] / 2 * E.ns[1] * E.ns[2] >= 16777216.0) return fail(err, "Ns^3 / 2 must be below 2^24");
        for (int i = 0; i < P->n_dirs; ++i) {
            const int d = P->dirs[i];
            for (int rv : P->r)
                if (rv < 1 || rv >= E.ns[d]) return fail(err, "every r must satisfy 1 <= r < Ns along the charge axis");
            for (const u1ml_probe& pr : P->probes) {
                const int n1 = E.ns[(d + 1) % 3], n2 = E.ns[(d + 2) % 3];
                if (std::abs(pr.p1) * 2 >= n1) return fail(err, "probe |p1| must be < Ns/2");
                if (std::abs(pr.p2) * 2 >= n2) return fail(err, "probe |p2| must be < Ns/2");
                if (std::abs(pr.l) >= E.ns[d]) return fail(err, "probe |l| must be < Ns along the charge axis");
                if (pr.mode != 0 && pr.mode != 1) return fail(err, "probe mode must be 0 or 1");
            }
        }
    }
    P->nd_cfg = 2ll * P->r.size() + 4ll * P->r.size() * P->probes.size() * P->comps.size() + 12 + P->r.size();
    if (p->form < U1ML_FORM_AUTO || p->form > U1ML_FORM_SPECTRAL) return fail(err, "form must be 0, 1 or 2");
    P->form_req = p->form;
    if (p->form == U1ML_FORM_SPECTRAL)
        for (const u1ml_ensemble& E : P->ens)
            for (int i = 0; i < P->n_dirs; ++i)
                if ((long long)E.ns[0] * E.ns[1] * E.ns[2] / E.ns[P->dirs[i]] > 4096)
                    return fail(err, "spectral form: a transverse plane has more than 4096 sites");
    // probes sharing (l, mode) share one longitudinal offset per (r, component)
    P->pgroup.clear();
    P->gdesc.clear();
    for (const u1ml_probe& pr : P->probes) {
        int g = 0;
        while (g < (int)P->gdesc.size() / 2 && !(P->gdesc[2 * g] == pr.l && P->gdesc[2 * g + 1] == pr.mode)) ++g;
        if (g == (int)P->gdesc.size() / 2) {
            P->gdesc.push_back(pr.l);
            P->gdesc.push_back(pr.mode);
        }
        P->pgroup.push_back(g);
    }
    // slot keys of the insertion contraction: the (probe, component) pairs
    // of each probe group whose plaquettes span the axis, then those whose
    // plaquettes do not (probes, then components, in problem order); blocks
    // of KS slots of one key, KS in {9, 6, 3, 1}, or kMfSlots for the
    // matrix-core kernel (the planner's choice, pack_slot_blocks)
    P->skeys.clear();
    P->skey_l.clear();
    P->skey_mode.clear();
    P->skey_spans.clear();
    for (int g = 0; g < (int)P->gdesc.size() / 2; ++g)
        for (int sp = 1; sp >= 0; --sp) {
            std::vector<std::pair<int, int>> slots;
            for (int p = 0; p < (int)P->probes.size(); ++p)
                if (P->pgroup[p] == g)
                    for (int ic = 0; ic < (int)P->comps.size(); ++ic)
                        if ((int)comp_spans_axis_host(P->comps[ic]) == sp) slots.emplace_back(p, ic);
            if (slots.empty()) continue;
            P->skeys.push_back(slots);
            P->skey_l.push_back(P->gdesc[2 * g]);
            P->skey_mode.push_back(P->gdesc[2 * g + 1]);
            P->skey_spans.push_back(sp);
        }
    // the block size whose padded work (slots rounded up to whole blocks,
    // separations to whole groups of ins_kr(KS)) is least; on a tie FP32 O
    // rows take the smaller block (each O value is converted to FP64 where it
    // is read, once per ins_kr(KS) separations: C2 FP32 11.51 ms per
    // configuration with blocks of 3 against 11.72 with 9) and FP64 rows the
    // larger (C2 FP64 16.80 ms with 9 against 17.05 with 3); blocks of 1 only
    // where they pad least (eight separations per work-item form more T)
    const size_t R_ = P->r.size();
    double best = 1e300;
    int best_ks = 1;
    const bool fp32_o = P->precision == U1ML_FP32;
    for (int ks : {9, 6, 3, 1}) {
        size_t padded = 0;
        for (const auto& k : P->skeys) padded += (k.size() + ks - 1) / ks * ks;
        const int kr = ins_kr(ks);
        const double work = (double)padded * (double)((R_ + kr - 1) / kr * kr);
        if (work < best || (fp32_o && work == best && ks >= 3)) {
            best = work;
            best_ks = ks;
        }
    }
    P->ins_ks_vec = best_ks;
    pack_slot_blocks(P, best_ks);
    return true;
}

// Kernel launches of one multilevel body (upper bound).  Bodies above
// kMaxGraphLaunches are launched directly instead of through one captured
// graph: a single capture of a full configuration of the largest preset
// (about 275,000 kernel nodes in one chain) ended the process with a
// segmentation fault, so graphs stay at the sizes that are tested.
constexpr long long kMaxGraphLaunches = 8192;

long long body_launches(const Problem& P)
{
    const long long sweep = (1ll + P.n_or) * 8;
    // per measurement: the measurement, and in the spectral form staging,
    // plane transforms and spectral sums (at most 6); per inner level: the two
    // contractions, the combine, the exponent pass (2) and the weights
    const long long meas = 1 + (P.spectral ? 6 : 0);
    const long long level = (long long)P.n_o * ((long long)P.k_o * sweep + (long long)P.n_i * (P.k_i * sweep + meas) + 6);
    const long long passes = (P.spectral && P.two) ? 2 : 1;
    // per configuration: products (4), vacuum, spectral final (2), outer
    // weights, ring and counters; per ensemble: up to three fills and two
    // link copies
    return passes * level + 10 + 5ll * P.n_ens;
}

// probe groups of the slab-product launch: every probe in the history form,
// one (the correlator only) otherwise; the work-group table, the partial
// buffer and the launch all use this count
int prod_groups(const Problem& P) { return (!P.spectral && !P.probes.empty()) ? (int)P.probes.size() : 1; }

bool compute_sizes(Problem& P, Sizes* S, u1ml_plan_info* info, Layout* Lo, std::string* err)
{
    const size_t word = P.precision == U1ML_FP64 ? 8 : 4;
    const bool store_o = !P.probes.empty();
    const size_t R = P.r.size(), Np = P.probes.size(), Nc = P.comps.size(), nd = (size_t)P.n_dirs;
    const size_t NG = P.gdesc.size() / 2;
    // contraction form: the spectral form needs every transverse plane of a
    // charge axis within 4096 sites.  AUTO estimates the device time each
    // form adds to a configuration and takes the smaller (history also when
    // the spectral form does not apply, spectral when the history form's
    // per-site averages would exceed 64 GiB); the unit costs are MI355X
    // measurements (FP32 links):
    //   history:  contraction 6.6e12 FMA/s (the inner level's [TO] sums,
    //             vector kernel) or 0.18 of the FP64 matrix-core peak per
    //             16 x 16 x 4 step, padding included (matrix-core kernel:
    //             3.3 ms per launch on the 24^3x8 workload below against 1.5 for the
    //             vector kernel; a plain stream of these steps runs at 46
    //             TFLOP/s on MI355X, FP64 vector FMA at 61);
    //             two levels: the inner averages folded into the outer sums,
    //             3 passes over them per outer update at 3 TB/s;
    //   spectral: per measurement 20 us of launches, 14.2 ps per plane
    //             element and field (staging and transforms), 0.198 ps per
    //             flop of the spectral sums; two levels: the replay repeats
    //             every update (5e10 link updates/s).
    // Measured per configuration (history / spectral, ms): 24^3x8, 9 probes,
    // 100 updates 11.5 / 18.0; 24^3x8 in-plane map 18.1 / 19.4; 48^3x12 two
    // levels 2 x 10, 1 probe 8.8 / 21.5, 8 probes 39.9 / 21.6.
    {
        bool plane_ok = true;
        double hist_avg = 0.0, est_h = 0.0, est_s = 0.0, est_v = 0.0, est_m = 0.0;
        const double n_meas = (double)P.n_i * (P.two ? P.n_o : 1);
        const double n_steps = (double)((P.n_i + 3) / 4) * (P.two ? P.n_o : 1);  // MFMA steps of 4 measurements
        size_t nblk8 = 0;
        for (const auto& k : P.skeys) nblk8 += (k.size() + kMfSlots - 1) / kMfSlots;
        const int word_o = P.precision == U1ML_FP64 ? 8 : 4;
        bool mf_ok = R <= (size_t)kMfR;
        for (const u1ml_ensemble& E : P.ens) {
            const double nsig = (double)E.ns[0] * E.ns[1] * E.ns[2];
            for (int i = 0; i < P.n_dirs; ++i)
                if (nsig / E.ns[P.dirs[i]] > 4096.0) plane_ok = false;
            const int nmax = std::max(E.ns[0], std::max(E.ns[1], E.ns[2]));  // as the contraction is sized
            if (!mf_chunk_fits(4, nmax, (int)R, 2 * kMfSlots, word_o)) mf_ok = false;
            const double per = (double)nd * R * Np * Nc * 2 * nsig * 16.0;
            const double si = (double)(E.nt / P.tau_i);
            hist_avg += per * si + (P.two ? per * (E.nt / P.tau_o) : 0.0);
            est_v += n_meas * nd * si * nsig * R * Np * Nc * 4.0 / 6.6e12;
            est_m += n_steps * nd * si * nsig * (double)((R + 7) / 8) * nblk8 * 1024.0 / (0.18 * 39.3e12);
            if (P.two) est_h += (double)P.n_o * per * si * 3.0 / 3.0e12;
            est_s += n_meas * (20e-6 + nd * si * nsig * (R + 12) * 14.2e-12 + nd * si * (double)NG * nsig * R * Nc * 16.0 * 0.198e-12);
            if (P.two) {
                const double V = nsig * E.nt, vh = V / 2;
                const double sp_i = vh / E.nt * (E.nt - E.nt / P.tau_i), sp_o = vh / E.nt * (E.nt - E.nt / P.tau_o);
                const double upd = (double)P.n_o * ((double)P.k_o * (1 + P.n_or) * 2 * (vh + 3 * sp_o) +
                                                    (double)P.n_i * P.k_i * (1 + P.n_or) * 2 * (vh + 3 * sp_i));
                est_s += upd / 5e10;
            }
        }
        P.ins_mfma_est = Np && (P.ins_kernel == 2 || (P.ins_kernel == 0 && mf_ok && est_m < est_v));
        est_h += P.ins_mfma_est ? est_m : est_v;
        P.est_hist_ms = Np ? est_h * 1e3 : 0.0;
        P.est_spec_ms = (Np && plane_ok) ? est_s * 1e3 : -1.0;
        if (P.form_req == U1ML_FORM_SPECTRAL) {
            P.spectral = !P.probes.empty();  // planes checked by read_problem
        } else if (P.form_req == U1ML_FORM_AUTO) {
            P.spectral = !P.probes.empty() && plane_ok &&
                         (est_s < est_h || hist_avg > 64.0 * 1024 * 1024 * 1024);
        } else {
            P.spectral = false;
        }
    }
    // slot blocks for the kernel that sums the history form
    if (Np && !P.spectral) {
        const int ks = P.ins_mfma_est ? kMfSlots : P.ins_ks_vec;
        if (P.ins_ks != ks) pack_slot_blocks(&P, ks);
    }
    const bool spec = P.spectral;
    size_t L = 0, HC = 0, HO = 0, AT = 0, ATO = 0, OT = 0, OTO = 0, VAC = 0, PP = 0;
    size_t maxV = 0, paper = 0, upd_cfg = 0, upd_sweep = 0, blocks64 = 0, mblocks = 0;
    S->links.clear();
    S->hc.clear();
    S->ho.clear();
    S->at.clear();
    S->ato.clear();
    S->ot.clear();
    S->oto.clear();
    S->vac.clear();
    S->wf.clear();
    S->gf.clear();
    S->sph.clear();
    S->spo.clear();
    S->facc.clear();
    S->cpl.clear();
    S->opl.clear();
    size_t WF = 0, GF = 0, SPH = 0, SPO = 0, FACC = 0, CPL = 0, OPL = 0;
    for (const u1ml_ensemble& E : P.ens) {
        const size_t nsig = (size_t)E.ns[0] * E.ns[1] * E.ns[2];
        const size_t V = nsig * E.nt;
        maxV = std::max(maxV, V);
        blocks64 += (V / 2 + 63) / 64;
        blocks64 += 8;  // padding of the XCD-aware block order
        const size_t si = E.nt / P.tau_i, so = E.nt / P.tau_o;
        size_t v, t;
        // links: 4 V words, padded to 256 bytes
        if (!mul_ok(4 * V, word, &v)) return fail(err, "size overflow (links)");
        S->links.push_back(L / word);
        L = align_up(L + v);
        S->hc.push_back(HC);
        // plain slab phases, then (multihit) the multihit ones
        if (!mul_ok((size_t)P.n_i * si * (P.multihit ? 2 : 1), nsig, &t) || !add_ok(HC, t, &HC))
            return fail(err, "size overflow (history)");
        HC = align_up(HC * 16) / 16;
        S->ho.push_back(HO);
        if (store_o) {
            if (!mul_ok((size_t)P.n_i * si * 12, nsig, &t) || !add_ok(HO, t, &HO)) return fail(err, "size overflow (history)");
            HO = align_up(HO * word) / word;
        }
        S->at.push_back(AT);
        AT = align_up((AT + nd * R * si * nsig) * 16) / 16;
        S->ato.push_back(ATO);
        if (store_o && !spec) {
            if (!mul_ok(nd * R * Np * Nc * 2 * si, nsig, &t) || !add_ok(ATO, t, &ATO)) return fail(err, "size overflow (averages)");
            ATO = align_up(ATO * 16) / 16;
        }
        S->ot.push_back(OT);
        S->oto.push_back(OTO);
        if (P.two) {
            OT = align_up((OT + nd * R * so * nsig) * 16) / 16;
            if (store_o && !spec) {
                if (!mul_ok(nd * R * Np * Nc * 2 * so, nsig, &t) || !add_ok(OTO, t, &OTO)) return fail(err, "size overflow (outer)");
                OTO = align_up(OTO * 16) / 16;
            }
        }
        S->wf.push_back(WF);
        S->gf.push_back(GF);
        S->sph.push_back(SPH);
        S->spo.push_back(SPO);
        S->facc.push_back(FACC);
        S->cpl.push_back(CPL);
        S->opl.push_back(OPL);
        if (spec) {
            CPL = align_up((CPL + nd * si * nsig) * 16) / 16;
            OPL = align_up((OPL + nd * si * 12 * nsig) * word) / word;
            size_t n12max = 0;
            for (int i = 0; i < P.n_dirs; ++i) n12max = std::max(n12max, nsig / (size_t)E.ns[P.dirs[i]]);
            if (P.two) WF = align_up((WF + nd * R * so * nsig) * 16) / 16;
            GF = align_up((GF + nd * R * si * nsig) * 16) / 16;
            SPH = align_up((SPH + nd * si * R * nsig) * 16) / 16;
            SPO = align_up((SPO + nd * si * 12 * nsig) * 16) / 16;
            if (!mul_ok(nd * si * R * Nc * 2 * NG, n12max, &t) || !add_ok(FACC, t, &FACC))
                return fail(err, "size overflow (spectral sums)");
            FACC = align_up(FACC * 16) / 16;
        }
        S->vac.push_back(VAC);
        // running double-double vacuum partials, one set of 12 per measurement block
        VAC += ((nsig * si + 255) / 256) * 24;
        // slab-product partials: per (r, probe group, site chunk) work-group
        PP += R * (size_t)prod_groups(P) * ((nd * nsig + kProdChunk - 1) / kProdChunk) * kProdQ * 2;
        mblocks += (nsig * si + 255) / 256;
        // the paper's running accumulators: 2 doubles per site and per point of
        // the transverse plane, per slab of the inner level (Sec. II.D)
        const size_t area = (size_t)E.ns[(P.dirs[0] + 1) % 3] * E.ns[(P.dirs[0] + 2) % 3];
        paper += 2 * 8 * V * area / P.tau_i;
        // link updates
        const size_t vh = V / 2;
        const size_t sp_i = vh / E.nt * (E.nt - E.nt / P.tau_i);  // spatial links of one parity, one direction
        const size_t sp_o = vh / E.nt * (E.nt - E.nt / P.tau_o);
        const size_t per_sweep_i = (1 + P.n_or) * 2 * (vh + 3 * sp_i);
        const size_t per_sweep_o = (1 + P.n_or) * 2 * (vh + 3 * sp_o);
        upd_cfg += (size_t)P.n_o * ((size_t)P.k_o * per_sweep_o + (size_t)P.n_i * P.k_i * per_sweep_i);
        upd_sweep += (1 + P.n_or) * 4 * V;
    }
    Lo->sz_links = align_up(L);
    Lo->sz_hc = align_up(HC * 16);
    Lo->sz_ho = align_up(HO * word);
    Lo->sz_at = align_up(AT * 16);
    Lo->sz_ato = align_up(ATO * 16);
    Lo->sz_ot = align_up(OT * 16);
    Lo->sz_oto = align_up(OTO * 16);
    Lo->sz_wf = align_up(WF * 16);
    Lo->sz_gf = align_up(GF * 16);
    Lo->sz_sph = align_up(SPH * 16);
    Lo->sz_spo = align_up(SPO * 16);
    Lo->sz_facc = align_up(FACC * 16);
    Lo->sz_cpl = align_up(CPL * 16);
    Lo->sz_opl = align_up(OPL * word);
    Lo->sz_saved = (spec && P.two) ? Lo->sz_links : 0;
    size_t res;
    if (!mul_ok((size_t)P.max_configs * P.n_ens, (size_t)P.nd_cfg * 8, &res)) return fail(err, "size overflow (results)");
    Lo->sz_res = align_up(res);
    // scratch
    size_t s = 0;
    auto take = [&](size_t bytes) {
        const size_t o = s;
        s = align_up(s + bytes);
        return o;
    };
    const int n = P.n_ens;
    Lo->s_ens = take(sizeof(EnsDesc) * n);
    Lo->s_obs = take(sizeof(ObsDesc));
    Lo->s_r = take(sizeof(int) * R);
    Lo->s_probe = take(sizeof(int) * 4 * std::max<size_t>(Np, 1));
    Lo->s_comp = take(sizeof(int) * std::max<size_t>(Nc, 1));
    Lo->n_bstart_tables = kNumTabs;
    Lo->s_bstart = take(sizeof(int) * (n + 1) * kNumTabs);
    Lo->s_upd = take(sizeof(uint32_t) * n);
    Lo->s_ring = take(sizeof(int) * 4);
    Lo->s_vpart = take(sizeof(double) * VAC);
    Lo->s_ppart = take(sizeof(double) * 6 * kPlaqBlocks * n);
    Lo->s_pout = take(sizeof(double) * 6 * n);
    Lo->s_count = take(sizeof(unsigned long long) * 2);
    Lo->s_stage = take(sizeof(double) * 4 * maxV);
    Lo->bmap_stride = blocks64;
    Lo->s_bmap = take(sizeof(UpdBlock) * kUpdateClasses * blocks64);
    Lo->s_mmap = take(sizeof(int2) * mblocks);
    Lo->s_prodpart = take(sizeof(double) * PP);
    for (int l = 0; l < kMaxLanes; ++l) {
        Lo->s_lens[l] = take(sizeof(EnsDesc) * n);
        Lo->s_lbstart[l] = take(sizeof(int) * (n + 1) * kNumTabs);
        Lo->s_lbmap[l] = take(sizeof(UpdBlock) * kUpdateClasses * blocks64);
        Lo->s_lmmap[l] = take(sizeof(int2) * mblocks);
        Lo->s_lring[l] = take(sizeof(int) * 4);
    }
    Lo->s_pgroup = take(sizeof(int) * std::max<size_t>(Np, 1));
    Lo->s_gdesc = take(sizeof(int) * std::max<size_t>(2 * NG, 2));
    Lo->s_pblk = take(sizeof(int) * std::max<size_t>(P.pblk.size(), kInsBlkInts));
    Lo->sz_scr = s;
    size_t off = 0;
    Lo->off_links = off;
    off += Lo->sz_links;
    Lo->off_hc = off;
    off += Lo->sz_hc;
    Lo->off_ho = off;
    off += Lo->sz_ho;
    Lo->off_at = off;
    off += Lo->sz_at;
    Lo->off_ato = off;
    off += Lo->sz_ato;
    Lo->off_ot = off;
    off += Lo->sz_ot;
    Lo->off_oto = off;
    off += Lo->sz_oto;
    Lo->off_res = off;
    off += Lo->sz_res;
    Lo->off_wf = off;
    off += Lo->sz_wf;
    Lo->off_gf = off;
    off += Lo->sz_gf;
    Lo->off_sph = off;
    off += Lo->sz_sph;
    Lo->off_spo = off;
    off += Lo->sz_spo;
    Lo->off_facc = off;
    off += Lo->sz_facc;
    Lo->off_saved = off;
    off += Lo->sz_saved;
    Lo->off_cpl = off;
    off += Lo->sz_cpl;
    Lo->off_opl = off;
    off += Lo->sz_opl;
    Lo->off_scr = off;
    off += Lo->sz_scr;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->ws_bytes = off;
        info->link_bytes = Lo->sz_links;
        info->history_bytes = Lo->sz_hc + Lo->sz_ho;
        info->average_bytes = Lo->sz_at + Lo->sz_ato;
        info->outer_bytes = Lo->sz_ot + Lo->sz_oto;
        info->result_bytes = Lo->sz_res;
        info->scratch_bytes = Lo->sz_scr;
        info->paper_running_bytes = paper;
        info->n_doubles_per_config = P.nd_cfg;
        info->updates_per_config = (long)upd_cfg;
        info->updates_per_sweep = (long)upd_sweep;
        info->form = spec ? U1ML_FORM_SPECTRAL : U1ML_FORM_HISTORY;
        info->spectral_bytes = Lo->sz_wf + Lo->sz_gf + Lo->sz_sph + Lo->sz_spo + Lo->sz_facc + Lo->sz_saved +
                               Lo->sz_cpl + Lo->sz_opl;
        info->launches_per_config = (long)body_launches(P);
        info->est_history_ms = P.est_hist_ms;
        info->est_spectral_ms = P.est_spec_ms;
        info->ins_slots = (!P.probes.empty() && !P.spectral) ? P.ins_ks : 0;
    }
    return true;
}

}  // namespace

// A lane: a subset of the problem's ensembles with its own descriptors,
// launch tables, results-ring counter, stream and graphs.  The whole batch
// is one lane (used by every call); a batch of two or more ensembles is also
// split into up to four lanes of about equal volume that run sweeps and
// multilevel configurations on as many streams at once.  A checkerboard
// phase of a few tens of MB lasts a few microseconds, most of it the latency
// of its dependent loads and of the launch itself, so phases of different
// lanes running side by side fill the machine where one alone does not, and
// the heatbath phases (bound by arithmetic) of one lane overlap the
// overrelaxation phases (bound by memory) of another.  Each ensemble's
// arithmetic is the same in every lane arrangement.
struct Lane {
    int n = 0;
    std::vector<int> idx;        // problem indices of the lane's ensembles
    std::vector<EnsDesc> h_ens;  // their descriptors, lane order
    std::vector<int> h_bstart;   // kNumTabs x (n + 1)
    std::vector<UpdBlock> h_bmap;  // per-block update records, kUpdateClasses x bmap_stride
    std::vector<int2> h_mmap;    // measurement block -> (lane ensemble, block)
    EnsDesc* d_ens = nullptr;
    int* d_bstart = nullptr;
    UpdBlock* d_bmap = nullptr;
    int2* d_mmap = nullptr;
    int* d_ring = nullptr;
    double* prodpart = nullptr;
    size_t bmap_stride = 0;
    int upd_grid[kUpdateClasses] = {0, 0, 0, 0};  // grid size of each update class (multiple of 8)
    int max_s_in = 1;                              // largest number of inner slabs in the lane
    hipStream_t stream = nullptr;
    hipGraphExec_t g_sweep = nullptr, g_ml = nullptr;

    int tab_total(int tab) const { return h_bstart[(size_t)tab * (n + 1) + n]; }
    const int* tab_dev(int tab) const { return d_bstart + (size_t)tab * (n + 1); }
    const UpdBlock* bmap_dev(int cls) const { return d_bmap + (size_t)cls * bmap_stride; }
};

struct u1ml_ctx {
    Problem P;
    Sizes S;
    Layout Lo;
    u1ml_plan_info plan;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    hipStream_t lane_stream[kMaxLanes] = {};  // streams of lanes 1.. (lane 0 runs on the context's stream)
    hipEvent_t ev_fork = nullptr, ev_join[kMaxLanes] = {};
    int device = 0;
    // device pointers
    void* links = nullptr;
    double2 *hc = nullptr, *at = nullptr, *ato = nullptr, *ot = nullptr, *oto = nullptr;
    void* ho = nullptr;
    double *res = nullptr, *vpart = nullptr, *ppart = nullptr, *pout = nullptr,
           *stage = nullptr;
    ObsDesc* d_obs = nullptr;
    int *d_r = nullptr, *d_probe = nullptr, *d_comp = nullptr;
    int con_block = 64;                            // contraction work-group size
    size_t con_lds = 0;                            // contraction dynamic LDS per work-group
    double2 *wf = nullptr, *gf = nullptr, *sph = nullptr, *spo = nullptr, *facc = nullptr;  // spectral form
    double2* cpl = nullptr;                        // plane-major slab phases of one measurement
    void* opl = nullptr;                           // plane-major O rows of one measurement
    void* saved = nullptr;                         // replay copy of the links
    int spec_npm = 0;                              // largest lattice extent (spectral launches)
    long long spec_n12max = 0;                     // largest transverse plane (sites)
    int spec_tile = 4;                             // plane-transform tile (4, or 2 if an extent is not a multiple of 4)
    int *d_pgroup = nullptr, *d_gdesc = nullptr, *d_pblk = nullptr;
    size_t ins_lds = 0;  // insertion contraction dynamic LDS per work-group
    int ins_block = 64;  // insertion contraction work-group size
    int ins_line_len = 0;  // sites of every charge-axis line of every ensemble where they are all the same, else 0
    uint32_t* d_upd = nullptr;
    unsigned long long* d_count = nullptr;
    double* static_partials = nullptr;  // the library's static scratch on this context's device
    std::vector<EnsDesc> h_ens;  // descriptors in problem order
    Lane whole;                  // every ensemble
    Lane split[kMaxLanes];       // the lanes (batches of two or more ensembles)
    int n_lanes = 1;             // lanes that sweeps and configurations run on (1: the whole batch)
    int block = 256;
    bool initialised = false;
    int ring_count = 0;
    bool use_graphs = true;
    std::string err;
};

namespace {

// the whole-batch lane and every lane of the split (those not in use have no ensembles)
std::vector<Lane*> all_lanes(u1ml_ctx* c)
{
    std::vector<Lane*> v{&c->whole};
    for (int l = 0; l < kMaxLanes; ++l) v.push_back(&c->split[l]);
    return v;
}

u1ml_status set_err(u1ml_ctx* c, u1ml_status s, const std::string& m)
{
    if (c)
        c->err = m;
    else
        g_err = m;
    return s;
}

#define HIPCHK(ctx, expr)                                                                                    \
    do {                                                                                                     \
        hipError_t _e = (expr);                                                                              \
        if (_e != hipSuccess)                                                                                \
            return set_err((ctx), U1ML_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));          \
    } while (0)

void build_tab(Lane& L, int tab, const std::vector<long long>& items, int block)
{
    int* b = &L.h_bstart[(size_t)tab * (L.n + 1)];
    b[0] = 0;
    for (int e = 0; e < L.n; ++e) b[e + 1] = b[e] + (int)((items[e] + block - 1) / block);
}

void build_update_tabs(const u1ml_ctx* c, Lane& L)
{
    const Problem& P = c->P;
    const int n = L.n;
    std::vector<long long> it0(n), it1(n), it2(n), it3(n);
    for (int e = 0; e < n; ++e) {
        const EnsDesc& E = L.h_ens[e];
        const long long slice = (long long)E.nxh * E.ny * E.nz;
        it0[e] = (long long)E.vh;
        it1[e] = (long long)E.vh;
        it2[e] = slice * (P.tau_i > 1 ? E.nt - E.nt / P.tau_i : E.nt);
        it3[e] = slice * (P.tau_o > 1 ? E.nt - E.nt / P.tau_o : E.nt);
    }
    build_tab(L, kTabUpd + 0, it0, c->block);
    build_tab(L, kTabUpd + 1, it1, c->block);
    build_tab(L, kTabUpd + 2, it2, c->block);
    build_tab(L, kTabUpd + 3, it3, c->block);
    // Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b mod 8),
    // and each XCD has its own L2.  Logical block L(b) = (b mod 8) per + b / 8
    // gives every XCD one contiguous stretch of the lattice, so neighbouring
    // rows shared by adjacent blocks are fetched into one L2 instead of
    // several.  Launches have 8 per blocks; entries past the end are idle.
    UpdBlock pad;
    std::memset(&pad, 0, sizeof pad);
    pad.e = -1;
    L.h_bmap.assign((size_t)kUpdateClasses * L.bmap_stride, pad);
    const std::vector<long long>* items[kUpdateClasses] = {&it0, &it1, &it2, &it3};
    for (int cls = 0; cls < kUpdateClasses; ++cls) {
        const int* b = &L.h_bstart[(size_t)(kTabUpd + cls) * (n + 1)];
        const int total = b[n];
        const int per = (total + kXcds - 1) / kXcds;
        std::vector<UpdBlock> logical(total);
        for (int e = 0; e < n; ++e) {
            const EnsDesc& E = L.h_ens[e];
            UpdBlock r = pad;
            r.e = e;
            r.nx = E.nx;
            r.ny = E.ny;
            r.nz = E.nz;
            r.nt = E.nt;
            r.nxh = E.nxh;
            r.vh = E.vh;
            r.inv_slice = E.inv_slice;
            r.inv_nxh = E.inv_nxh;
            r.inv_ny = E.inv_ny;
            r.res_index = E.res_index;
            r.link_off = E.link_off;
            r.n_items = (int)(*items[cls])[e];
            // Time slice fastest: when a slice of sites is a whole number of
            // blocks, the blocks of one stretch of the slice at consecutive
            // times follow each other, so the links a slice shares with the
            // next one are reused while they are still in the XCD's L2.
            const int nb = b[e + 1] - b[e];
            const long long slice = (long long)E.nxh * E.ny * E.nz;
            const int bps = slice % c->block == 0 ? (int)(slice / c->block) : 0;
            const int ns = bps > 0 ? nb / bps : 0;
            for (int k = 0; k < nb; ++k) {
                r.blk = (ns > 1 && ns * bps == nb) ? (k % ns) * bps + k / ns : k;
                logical[b[e] + k] = r;
            }
        }
        // padding blocks: the last ensemble's record with a block index past
        // its links (every work-item inactive)
        UpdBlock idle = total > 0 ? logical[total - 1] : pad;
        idle.blk = total > 0 ? b[n] - b[n - 1] : 0;
        for (int phys = 0; phys < per * kXcds; ++phys) {
            const int lg = (phys % kXcds) * per + phys / kXcds;
            L.h_bmap[(size_t)cls * L.bmap_stride + phys] = lg < total ? logical[lg] : idle;
        }
        L.upd_grid[cls] = per * kXcds;
    }
}

// Every launch table of a lane, from its ensembles' descriptors (whose
// contraction and product fields are already set).
void build_lane_tables(const u1ml_ctx* c, Lane& L)
{
    const Problem& P = c->P;
    const int n = L.n;
    L.h_bstart.assign((size_t)kNumTabs * (n + 1), 0);
    build_update_tabs(c, L);
    const size_t R = P.r.size(), NG = P.gdesc.size() / 2;
    std::vector<long long> all(n), meas(n), con(n), comb(n), prod(n), site(n), plane(n), mac(n), stage(n), ins(n);
    L.max_s_in = 1;
    for (int e = 0; e < n; ++e) {
        const EnsDesc& E = L.h_ens[e];
        const int n3[3] = {E.nx, E.ny, E.nz};
        int lines = 0;
        long long n12max = 0;
        for (int i = 0; i < P.n_dirs; ++i) {
            lines = std::max(lines, E.nsig / n3[P.dirs[i]]);
            n12max = std::max<long long>(n12max, E.nsig / n3[P.dirs[i]]);
        }
        const long long npm = std::max(E.nx, std::max(E.ny, E.nz));
        all[e] = 8ll * E.vh;
        meas[e] = (long long)E.nsig * E.s_in;
        con[e] = (lines + E.con_lpb - 1) / E.con_lpb;
        // insertion contraction: (line, slot-block chunk) work-groups of the axis with the most lines
        ins[e] = (!P.probes.empty() && !P.spectral)
                     ? (long long)lines * ((P.pblk.size() / kInsBlkInts + E.ins_pbw - 1) / E.ins_pbw)
                     : 0;
        comb[e] = (long long)P.n_dirs * R * E.s_out * E.nsig;
        prod[e] = (long long)R * prod_groups(P) * E.prod_nch;
        site[e] = (long long)P.n_dirs * R * E.nsig;
        plane[e] = P.spectral ? (long long)P.n_dirs * E.s_in * ((long long)R + 12) * npm : 0;
        mac[e] = P.spectral ? (long long)P.n_dirs * E.s_in * NG * ((n12max + kMacK - 1) / kMacK) : 0;
        // staging: work-groups of 32 x 32 tiles per (axis, slab), as k_plane_stage decodes them
        stage[e] = P.spectral ? (long long)P.n_dirs * E.s_in * ((E.nx + 31) / 32) * ((npm + 31) / 32) * npm : 0;
        L.max_s_in = std::max(L.max_s_in, E.s_in);
    }
    build_tab(L, kTabAll, all, 256);
    build_tab(L, kTabMeas, meas, 256);
    build_tab(L, kTabCon, con, 1);
    build_tab(L, kTabComb, comb, 256);
    build_tab(L, kTabProd, prod, 1);
    build_tab(L, kTabSite, site, 256);
    build_tab(L, kTabPlane, plane, 1);
    build_tab(L, kTabMac, mac, 1);
    build_tab(L, kTabStage, stage, 1);
    build_tab(L, kTabIns, ins, 1);
    L.h_mmap.clear();
    const int* b = &L.h_bstart[(size_t)kTabMeas * (n + 1)];
    for (int e = 0; e < n; ++e)
        for (int k = b[e]; k < b[e + 1]; ++k) L.h_mmap.push_back(make_int2(e, k - b[e]));
}

hipError_t upload_lane(const Lane& L)
{
    const int ring0[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpy(L.d_ens, L.h_ens.data(), sizeof(EnsDesc) * L.n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(L.d_bstart, L.h_bstart.data(), sizeof(int) * L.h_bstart.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(L.d_bmap, L.h_bmap.data(), sizeof(UpdBlock) * L.h_bmap.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !L.h_mmap.empty())
        e = hipMemcpy(L.d_mmap, L.h_mmap.data(), sizeof(int2) * L.h_mmap.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(L.d_ring, ring0, sizeof ring0, hipMemcpyHostToDevice);
    return e;
}

// Splits the batch into nl lanes of about equal volume (largest ensembles
// first, each to the lane with the least volume so far; a lane keeps the
// problem order), builds and uploads their tables.  Lanes past nl are
// emptied; their device areas stay reserved.
hipError_t split_lanes(u1ml_ctx* c, int nl)
{
    const int n = c->P.n_ens;
    const Layout& Lo = c->Lo;
    char* s = c->ws + Lo.off_scr;
    std::vector<int> order(n);
    for (int e = 0; e < n; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c->h_ens[a].vh > c->h_ens[b].vh; });
    std::vector<std::vector<int>> parts(nl);
    std::vector<long long> load(nl, 0);
    for (int e : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        parts[l].push_back(e);
        load[l] += c->h_ens[e].vh;
    }
    size_t pp_off = 0;
    for (int l = 0; l < kMaxLanes; ++l) {
        Lane& L = c->split[l];
        if (L.g_sweep) (void)hipGraphExecDestroy(L.g_sweep);
        if (L.g_ml) (void)hipGraphExecDestroy(L.g_ml);
        L.g_sweep = L.g_ml = nullptr;
        L.idx = l < nl ? parts[l] : std::vector<int>();
        std::sort(L.idx.begin(), L.idx.end());
        L.n = (int)L.idx.size();
        L.h_ens.clear();
        for (int e : L.idx) L.h_ens.push_back(c->h_ens[e]);
        L.bmap_stride = Lo.bmap_stride;
        L.d_ens = (EnsDesc*)(s + Lo.s_lens[l]);
        L.d_bstart = (int*)(s + Lo.s_lbstart[l]);
        L.d_bmap = (UpdBlock*)(s + Lo.s_lbmap[l]);
        L.d_mmap = (int2*)(s + Lo.s_lmmap[l]);
        L.d_ring = (int*)(s + Lo.s_lring[l]);
        // the lanes use disjoint parts of the slab-product partials
        L.prodpart = (double*)(s + Lo.s_prodpart) + pp_off;
        L.stream = l == 0 ? c->stream : c->lane_stream[l];
        if (L.n == 0) continue;
        build_lane_tables(c, L);
        pp_off += (size_t)L.tab_total(kTabProd) * kProdQ * 2;
        hipError_t e = upload_lane(L);
        if (e != hipSuccess) return e;
    }
    c->n_lanes = nl;
    return hipSuccess;
}

// Bytes [begin, end) of ensemble k's share of a section whose per-ensemble
// element offsets are off[] (elements of `elem` bytes, `total` bytes in all).
void ens_range(const std::vector<size_t>& off, int k, size_t elem, size_t total, size_t* begin, size_t* end)
{
    *begin = off[k] * elem;
    *end = k + 1 < (int)off.size() ? off[k + 1] * elem : total;
}

// Fill with zeros the shares of the lane's ensembles (a whole-array fill
// would race with the other lane).
hipError_t zero_lane(const Lane& L, void* base, const std::vector<size_t>& off, size_t elem, size_t total,
                     hipStream_t st)
{
    for (int e = 0; e < L.n; ++e) {
        size_t b, en;
        ens_range(off, L.idx[e], elem, total, &b, &en);
        hipError_t r = launch_fill_zero((char*)base + b, en - b, st);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

int update_class(const u1ml_ctx* c, int mu, int tau, bool* ok)
{
    *ok = true;
    if (mu == 3) return 0;
    if (tau <= 1) return 1;
    if (tau == c->P.tau_i) return 2;
    if (tau == c->P.tau_o) return 3;
    *ok = false;
    return -1;
}

hipError_t enq_phase(u1ml_ctx* c, const Lane& L, hipStream_t st, int kind, int mu, int parity, int tau,
                     int pass_offset, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr)
{
    bool ok;
    const int cls = update_class(c, mu, tau, &ok);
    if (!ok) return hipErrorInvalidValue;
    return launch_update(L.d_ens, L.bmap_dev(cls), L.upd_grid[cls], c->block, c->P.precision, c->links, c->d_upd,
                         pass_offset, kind, mu, parity, (mu < 3 && tau > 1) ? tau : 0, st, ev_start, ev_stop);
}

hipError_t enq_pass(u1ml_ctx* c, const Lane& L, hipStream_t st, int kind, int tau, int pass_offset)
{
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
            hipError_t e = enq_phase(c, L, st, kind, mu, p, tau, pass_offset);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

// one sweep: stochastic pass (heatbath or Metropolis) with counter offset hb,
// then n_or overrelaxation passes
hipError_t enq_sweep(u1ml_ctx* c, const Lane& L, hipStream_t st, int tau, int hb)
{
    const int stoch = c->P.update == U1ML_UPDATE_METROPOLIS ? U1ML_METROPOLIS : U1ML_HEATBATH;
    hipError_t e = enq_pass(c, L, st, stoch, tau, hb);
    for (int k = 0; e == hipSuccess && k < c->P.n_or; ++k) e = enq_pass(c, L, st, U1ML_OVERRELAX, tau, hb);
    return e;
}

// The n_o outer iterations of Algorithm 1 (one iteration for one level).
//   store_o:  measurements keep the slab sums of O
//   ins_hist: history form: per-site insertion averages, combined per level
//   spec_acc: spectral form: after each inner level, weights G_k and the
//             plane transforms of every stored measurement into the sums
// *hb returns the number of heatbath counter offsets used.
hipError_t enq_levels(u1ml_ctx* c, const Lane& L, hipStream_t st, bool store_o, bool ins_hist, bool spec_acc,
                      int* hb_out)
{
    const Problem& P = c->P;
    const int n = L.n;
    hipError_t e = hipSuccess;
    if (P.two && !spec_acc) {
        e = zero_lane(L, c->ot, c->S.ot, 16, c->Lo.sz_ot, st);
        if (e == hipSuccess && ins_hist) e = zero_lane(L, c->oto, c->S.oto, 16, c->Lo.sz_oto, st);
    }
    int hb = 0;
    for (int ko = 0; e == hipSuccess && ko < P.n_o; ++ko) {
        if (P.two)
            for (int k = 0; e == hipSuccess && k < P.k_o; ++k) e = enq_sweep(c, L, st, P.tau_o, hb++);
        for (int m = 0; e == hipSuccess && m < P.n_i; ++m) {
            for (int k = 0; e == hipSuccess && k < P.k_i; ++k) e = enq_sweep(c, L, st, P.tau_i, hb++);
            if (e == hipSuccess)
                e = launch_measure(L.d_ens, L.d_mmap, L.tab_total(kTabMeas), P.precision, c->links, c->hc, c->ho,
                                   c->vpart, m, ko * P.n_i + m, P.tau_i, store_o ? 1 : 0, P.multihit ? 1 : 0, st);
        }
        if (e == hipSuccess)
            e = launch_contract(L.d_ens, L.tab_dev(kTabCon), n, L.tab_total(kTabCon), c->con_block, c->con_lds,
                                c->d_obs, c->d_r, c->hc, c->at, P.n_i, L.max_s_in, P.n_dirs, st);
        if (e == hipSuccess && ins_hist)
            e = launch_contract_ins(L.d_ens, L.tab_dev(kTabIns), n, L.tab_total(kTabIns), c->ins_block, c->ins_lds,
                                    c->d_obs, c->d_r, c->d_comp, c->d_pblk, P.ins_ks, c->hc, c->ho, c->ato, P.n_i,
                                    P.precision, L.max_s_in, P.n_dirs, c->ins_line_len, st);
        if (e == hipSuccess && P.two && !spec_acc)
            e = launch_combine(L.d_ens, L.tab_dev(kTabComb), n, L.tab_total(kTabComb), c->d_obs, c->at,
                               ins_hist ? c->ato : nullptr, c->ot, ins_hist ? c->oto : nullptr, P.tau_o / P.tau_i, st);
        if (spec_acc) {
            // one level: the weights are relative to 2^E(r) of this level's correlator products
            if (e == hipSuccess && !P.two)
                e = launch_prod_exp(L.d_ens, L.tab_dev(kTabProd), n, L.tab_total(kTabProd), c->d_obs,
                                    (int)P.r.size(), prod_groups(P), c->at, 0, 1.0, L.prodpart, c->res, L.d_ring, st);
            if (e == hipSuccess)
                e = launch_gfac(L.d_ens, L.tab_dev(kTabSite), n, L.tab_total(kTabSite), c->d_obs, c->at,
                                P.two ? c->wf : nullptr, P.two ? P.tau_o / P.tau_i : 0, c->gf, c->res, L.d_ring, st);
            const size_t lds = (2 * (size_t)c->spec_n12max + 2 * (size_t)c->spec_npm) * sizeof(double2);
            for (int m = 0; e == hipSuccess && m < P.n_i; ++m) {
                e = launch_plane_stage(L.d_ens, L.tab_dev(kTabStage), n, L.tab_total(kTabStage), c->d_obs, c->hc,
                                       c->ho, m, P.precision, c->cpl, c->opl, st);
                if (e == hipSuccess)
                    e = launch_dft_planes(L.d_ens, L.tab_dev(kTabPlane), n, L.tab_total(kTabPlane), lds, c->d_obs,
                                          c->d_r, c->cpl, c->opl, c->gf, c->sph, c->spo, P.precision,
                                          c->spec_tile, st);
                if (e == hipSuccess)
                    e = launch_spec_mac(L.d_ens, L.tab_dev(kTabMac), n, L.tab_total(kTabMac), c->spec_npm, c->d_obs,
                                        c->d_r, c->d_comp, c->d_gdesc, c->sph, c->spo, c->facc, st);
            }
        }
    }
    *hb_out = hb;
    return e;
}

// copies the links of the lane's ensembles (replay of two-level spectral configurations)
hipError_t copy_lane_links(u1ml_ctx* c, const Lane& L, const void* src, void* dst, hipStream_t st)
{
    const size_t word = c->P.precision == U1ML_FP64 ? 8 : 4;
    for (int e = 0; e < L.n; ++e) {
        size_t b, en;
        ens_range(c->S.links, L.idx[e], word, c->Lo.sz_links, &b, &en);
        hipError_t r = launch_copy((const char*)src + b, (char*)dst + b, en - b, st);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

// Body of Algorithm 1 for one configuration of the lane's ensembles.
//  history form: one pass; per-site averages of every probe, then products.
//  spectral form, one level: one pass; after the level the weights
//    W_s = prod_{s' != s} [T] are known and the stored measurements are
//    transformed into the spectral sums.
//  spectral form, two levels: pass 1 computes the correlator, the vacuum
//    sums and the outer averages A (no insertions); the links are restored
//    to the configuration's start and pass 2 repeats the same updates with
//    the same counters (so the same trajectory, bit for bit), forming the
//    spectral sums with G_k = W_S prod [T]_k after every inner level.
hipError_t enq_multilevel(u1ml_ctx* c, const Lane& L, hipStream_t st)
{
    const Problem& P = c->P;
    const int n = L.n;
    const bool probes = !P.probes.empty();
    const int npg = prod_groups(P);
    const int R = (int)P.r.size();
    hipError_t e = hipSuccess;
    int hb = 0;
    auto product = [&](bool ins) {  // ins only in the history form, where npg = number of probes
        if (P.two)
            return launch_product(L.d_ens, L.tab_dev(kTabProd), n, L.tab_total(kTabProd), c->d_obs, R, npg, c->ot,
                                  ins ? c->oto : nullptr, 1, 1.0 / P.n_o, L.prodpart, c->res, L.d_ring, st);
        return launch_product(L.d_ens, L.tab_dev(kTabProd), n, L.tab_total(kTabProd), c->d_obs, R, npg, c->at,
                              ins ? c->ato : nullptr, 0, 1.0, L.prodpart, c->res, L.d_ring, st);
    };
    const long long n_out = (long long)R * P.probes.size() * P.comps.size() * 2;
    if (!P.spectral) {
        e = enq_levels(c, L, st, probes, probes, false, &hb);
        if (e == hipSuccess) e = product(probes);
        if (e == hipSuccess) e = launch_vac_final(L.d_ens, n, c->d_obs, c->vpart, P.n_o * P.n_i, c->res, L.d_ring, st);
    } else if (!P.two) {
        e = zero_lane(L, c->facc, c->S.facc, 16, c->Lo.sz_facc, st);
        if (e == hipSuccess) e = enq_levels(c, L, st, true, false, true, &hb);
        if (e == hipSuccess) e = product(false);
        if (e == hipSuccess)
            e = launch_spec_final(L.d_ens, n, c->d_obs, n_out, c->spec_npm, c->d_probe, c->d_pgroup, c->facc,
                                  (double)P.n_i, c->res, L.d_ring, st);
        if (e == hipSuccess) e = launch_vac_final(L.d_ens, n, c->d_obs, c->vpart, P.n_i, c->res, L.d_ring, st);
    } else {
        e = copy_lane_links(c, L, c->links, c->saved, st);
        if (e == hipSuccess) e = enq_levels(c, L, st, false, false, false, &hb);
        if (e == hipSuccess) e = product(false);
        if (e == hipSuccess) e = launch_vac_final(L.d_ens, n, c->d_obs, c->vpart, P.n_o * P.n_i, c->res, L.d_ring, st);
        if (e == hipSuccess)
            e = launch_wfac(L.d_ens, L.tab_dev(kTabSite), n, L.tab_total(kTabSite), c->d_obs, c->ot, 1.0 / P.n_o,
                            c->wf, c->res, L.d_ring, st);
        if (e == hipSuccess) e = copy_lane_links(c, L, c->saved, c->links, st);
        if (e == hipSuccess) e = zero_lane(L, c->facc, c->S.facc, 16, c->Lo.sz_facc, st);
        int hb2 = 0;
        if (e == hipSuccess) e = enq_levels(c, L, st, true, false, true, &hb2);
        if (e == hipSuccess)
            e = launch_spec_final(L.d_ens, n, c->d_obs, n_out, c->spec_npm, c->d_probe, c->d_pgroup, c->facc,
                                  (double)P.n_o * P.n_i, c->res, L.d_ring, st);
    }
    if (e == hipSuccess) e = launch_ring_advance(L.d_ring, st);
    if (e == hipSuccess && hb > 0) e = launch_advance_counters(L.d_ens, c->d_upd, n, hb, st);
    return e;
}

hipError_t enq_sweep_with_counter(u1ml_ctx* c, const Lane& L, hipStream_t st)
{
    hipError_t e = enq_sweep(c, L, st, 0, 0);
    if (e == hipSuccess) e = launch_advance_counters(L.d_ens, c->d_upd, L.n, 1, st);
    return e;
}

void drop_graphs(u1ml_ctx* c)
{
    for (Lane* L : all_lanes(c)) {
        if (L->g_sweep) (void)hipGraphExecDestroy(L->g_sweep);
        if (L->g_ml) (void)hipGraphExecDestroy(L->g_ml);
        L->g_sweep = L->g_ml = nullptr;
    }
}

// graphs, streams and events of a context, then the context
void release(u1ml_ctx* c)
{
    drop_graphs(c);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    for (int l = 0; l < kMaxLanes; ++l) {
        if (c->ev_join[l]) (void)hipEventDestroy(c->ev_join[l]);
        if (c->lane_stream[l]) (void)hipStreamDestroy(c->lane_stream[l]);
    }
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
}

// Runs body(lane) for the lanes in use, all at once: the streams of lanes
// 1.. wait for the context's stream (lane 0's), and the context's stream
// waits for each of them at the end.  One lane: the whole batch on the
// context's stream.
template <typename F>
hipError_t on_lanes(u1ml_ctx* c, F&& body)
{
    if (c->n_lanes <= 1) return body(c->whole);
    hipError_t e = hipEventRecord(c->ev_fork, c->stream);
    for (int l = 1; l < c->n_lanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(c->lane_stream[l], c->ev_fork, 0);
    for (int l = 0; l < c->n_lanes && e == hipSuccess; ++l) e = body(c->split[l]);
    // the joins are enqueued whatever happened, so no lane stream is left behind
    for (int l = 1; l < c->n_lanes; ++l) {
        hipError_t j = hipEventRecord(c->ev_join[l], c->lane_stream[l]);
        if (j == hipSuccess) j = hipStreamWaitEvent(c->stream, c->ev_join[l], 0);
        if (e == hipSuccess) e = j;
    }
    return e;
}

template <typename F>
u1ml_status capture(u1ml_ctx* c, F&& body, hipGraphExec_t* out)
{
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
    hipError_t e = body(c->cap);
    hipError_t e2 = hipStreamEndCapture(c->cap, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return set_err(c, U1ML_EDEVICE, std::string("kernel launch during capture: ") + hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return set_err(c, U1ML_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return set_err(c, U1ML_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    return U1ML_OK;
}

// Streaming-model byte count of one phase: distinct words read + words written.
void phase_words(const u1ml_ensemble& E, int kind, int mu, int parity, int tau, long long* words, long long* updates)
{
    const int n[4] = {E.ns[0], E.ns[1], E.ns[2], E.nt};
    const long long V = (long long)n[0] * n[1] * n[2] * n[3];
    std::vector<unsigned char> rd((size_t)(4 * V), 0);
    long long w = 0, u = 0;
    auto sid = [&](int c[4]) { return (long long)c[0] + n[0] * ((long long)c[1] + n[1] * ((long long)c[2] + (long long)n[2] * c[3])); };
    for (int t = 0; t < n[3]; ++t)
        for (int z = 0; z < n[2]; ++z)
            for (int y = 0; y < n[1]; ++y)
                for (int x = 0; x < n[0]; ++x) {
                    if (((x + y + z + t) & 1) != parity) continue;
                    if (mu < 3 && tau > 1 && t % tau == 0) continue;
                    ++u;
                    int c[4] = {x, y, z, t};
                    if (kind != 0) rd[(size_t)(mu + 4 * sid(c))] = 1;
                    for (int nu = 0; nu < 4; ++nu) {
                        if (nu == mu) continue;
                        int a[4], b[4], d[4], f[4];
                        std::memcpy(a, c, sizeof a);
                        a[mu] = (a[mu] + 1) % n[mu];  // x + mu
                        std::memcpy(b, c, sizeof b);
                        b[nu] = (b[nu] + 1) % n[nu];  // x + nu
                        std::memcpy(d, c, sizeof d);
                        d[nu] = (d[nu] - 1 + n[nu]) % n[nu];  // x - nu
                        std::memcpy(f, a, sizeof f);
                        f[nu] = (f[nu] - 1 + n[nu]) % n[nu];  // x + mu - nu
                        rd[(size_t)(nu + 4 * sid(a))] = 1;
                        rd[(size_t)(mu + 4 * sid(b))] = 1;
                        rd[(size_t)(nu + 4 * sid(c))] = 1;
                        rd[(size_t)(nu + 4 * sid(d))] = 1;
                        rd[(size_t)(nu + 4 * sid(f))] = 1;
                        rd[(size_t)(mu + 4 * sid(d))] = 1;
                    }
                }
    for (unsigned char v : rd) w += v;
    *words = w + u;
    *updates = u;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* u1ml_status_str(u1ml_status s)
{
    switch (s) {
    case U1ML_OK: return "ok";
    case U1ML_EINVAL: return "invalid argument";
    case U1ML_ENOMEM: return "size overflow or out of host memory";
    case U1ML_EDEVICE: return "HIP device error";
    case U1ML_ESTATE: return "call made in the wrong state";
    case U1ML_ENOTSUP: return "not supported";
    }
    return "unknown status";
}

const char* u1ml_last_error(const u1ml_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

u1ml_status u1ml_plan(const u1ml_problem* problem, u1ml_plan_info* out)
{
    if (!out) return set_err(nullptr, U1ML_EINVAL, "plan output is NULL");
    Problem P;
    std::string err;
    if (!read_problem(problem, &P, &err)) return set_err(nullptr, U1ML_EINVAL, err);
    Sizes S;
    Layout Lo;
    if (!compute_sizes(P, &S, out, &Lo, &err)) return set_err(nullptr, U1ML_ENOMEM, err);
    g_err.clear();
    return U1ML_OK;
}

u1ml_status u1ml_create(const u1ml_problem* problem, void* d_ws, size_t ws_bytes, void* hip_stream, u1ml_ctx** out)
{
    if (!out) return set_err(nullptr, U1ML_EINVAL, "output pointer is NULL");
    *out = nullptr;
    u1ml_ctx* c = new (std::nothrow) u1ml_ctx();
    if (!c) return set_err(nullptr, U1ML_ENOMEM, "host allocation failed");
    std::string err;
    if (!read_problem(problem, &c->P, &err)) {
        delete c;
        return set_err(nullptr, U1ML_EINVAL, err);
    }
    if (!compute_sizes(c->P, &c->S, &c->plan, &c->Lo, &err)) {
        delete c;
        return set_err(nullptr, U1ML_ENOMEM, err);
    }
    if (!d_ws || ws_bytes < c->plan.ws_bytes) {
        const size_t need = c->plan.ws_bytes;
        delete c;
        return set_err(nullptr, U1ML_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    }
    if (((uintptr_t)d_ws) % kAlign != 0) {
        delete c;
        return set_err(nullptr, U1ML_EINVAL, "workspace must be 256-byte aligned");
    }
    c->ws = (char*)d_ws;
    c->stream = (hipStream_t)hip_stream;
    hipError_t he = hipGetDevice(&c->device);
    if (he == hipSuccess) he = static_scratch(&c->static_partials);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (he != hipSuccess) {
        delete c;
        return set_err(nullptr, U1ML_EDEVICE, std::string("stream creation: ") + hipGetErrorString(he));
    }
    const Layout& Lo = c->Lo;
    char* w = c->ws;
    c->links = w + Lo.off_links;
    c->hc = (double2*)(w + Lo.off_hc);
    c->ho = (void*)(w + Lo.off_ho);
    c->at = (double2*)(w + Lo.off_at);
    c->ato = (double2*)(w + Lo.off_ato);
    c->ot = (double2*)(w + Lo.off_ot);
    c->oto = (double2*)(w + Lo.off_oto);
    c->res = (double*)(w + Lo.off_res);
    char* s = w + Lo.off_scr;
    c->d_obs = (ObsDesc*)(s + Lo.s_obs);
    c->d_r = (int*)(s + Lo.s_r);
    c->d_probe = (int*)(s + Lo.s_probe);
    c->d_comp = (int*)(s + Lo.s_comp);
    c->d_upd = (uint32_t*)(s + Lo.s_upd);
    c->vpart = (double*)(s + Lo.s_vpart);
    c->ppart = (double*)(s + Lo.s_ppart);
    c->pout = (double*)(s + Lo.s_pout);
    c->d_count = (unsigned long long*)(s + Lo.s_count);
    c->stage = (double*)(s + Lo.s_stage);
    c->d_pgroup = (int*)(s + Lo.s_pgroup);
    c->d_gdesc = (int*)(s + Lo.s_gdesc);
    c->d_pblk = (int*)(s + Lo.s_pblk);
    c->wf = (double2*)(w + Lo.off_wf);
    c->gf = (double2*)(w + Lo.off_gf);
    c->sph = (double2*)(w + Lo.off_sph);
    c->spo = (double2*)(w + Lo.off_spo);
    c->facc = (double2*)(w + Lo.off_facc);
    c->cpl = (double2*)(w + Lo.off_cpl);
    c->opl = (void*)(w + Lo.off_opl);
    c->saved = (void*)(w + Lo.off_saved);

    const Problem& P = c->P;
    const int n = P.n_ens;
    c->h_ens.resize(n);
    for (int e = 0; e < n; ++e) {
        const u1ml_ensemble& U = P.ens[e];
        EnsDesc& E = c->h_ens[e];
        std::memset(&E, 0, sizeof E);
        E.nx = U.ns[0];
        E.ny = U.ns[1];
        E.nz = U.ns[2];
        E.nt = U.nt;
        E.nxh = E.nx / 2;
        E.nsig = E.nx * E.ny * E.nz;
        E.vh = E.nsig * E.nt / 2;
        E.s_in = E.nt / P.tau_i;
        E.s_out = P.two ? E.nt / P.tau_o : E.s_in;
        E.n_vac_blocks = (E.nsig * E.s_in + 255) / 256;
        E.inv_nxh = 1.0f / (float)E.nxh;
        E.inv_ny = 1.0f / (float)E.ny;
        E.inv_slice = 1.0f / (float)(E.nxh * E.ny * E.nz);
        E.beta = U.beta;
        E.sqrt_beta = std::sqrt(U.beta);
        E.metro_delta = P.metro_delta;
        E.seed = U.seed;
        E.key_id = U.key_id;
        E.link_off = (long long)c->S.links[e];
        E.hc_off = (long long)c->S.hc[e];
        E.hcm_off = E.hc_off + (long long)P.n_i * E.s_in * E.nsig;
        E.ho_off = (long long)c->S.ho[e];
        E.at_off = (long long)c->S.at[e];
        E.ato_off = (long long)c->S.ato[e];
        E.ot_off = (long long)c->S.ot[e];
        E.oto_off = (long long)c->S.oto[e];
        E.vac_part_off = (long long)c->S.vac[e];
        E.wf_off = (long long)c->S.wf[e];
        E.gf_off = (long long)c->S.gf[e];
        E.sph_off = (long long)c->S.sph[e];
        E.spo_off = (long long)c->S.spo[e];
        E.facc_off = (long long)c->S.facc[e];
        E.cpl_off = (long long)c->S.cpl[e];
        E.opl_off = (long long)c->S.opl[e];
    }
    ObsDesc O;
    std::memset(&O, 0, sizeof O);
    O.n_dirs = P.n_dirs;
    for (int i = 0; i < 3; ++i) O.dirs[i] = P.dirs[i];
    O.n_r = (int)P.r.size();
    O.n_probe = (int)P.probes.size();
    O.n_comp = (int)P.comps.size();
    O.store_o = P.probes.empty() ? 0 : 1;
    O.n_groups = (int)(P.gdesc.size() / 2);
    O.n_pblocks = (int)(P.pblk.size() / kInsBlkInts);
    O.n_ens_total = n;
    O.multihit = P.multihit ? 1 : 0;
    O.n_doubles_per_config = P.nd_cfg;
    std::vector<int> probe_flat;
    for (const u1ml_probe& p : P.probes) {
        probe_flat.push_back(p.l);
        probe_flat.push_back(p.p1);
        probe_flat.push_back(p.p2);
        probe_flat.push_back(p.mode);
    }
    // Contraction shape: a line of N sites along a charge axis has N * n_r
    // pairs (x, r), one thread each; a work-group of con_block threads holds
    // con_lpb such lines, and stages con_mc measurements at a time in LDS.
    // Insertions: a work-group per (line, slab, axis, ins_pbw slot blocks)
    // with N * ceil(n_r / KR) * ins_pbw tasks, staging ins_mc measurements
    // (the line's phases and the O rows of its slots).
    const size_t R = P.r.size();
    const size_t word = P.precision == U1ML_FP64 ? 8 : 4;  // O history element
    std::vector<int> group(n);
    c->con_block = 256;
    for (int e = 0; e < n; ++e) {
        const EnsDesc& E = c->h_ens[e];
        const int n3[3] = {E.nx, E.ny, E.nz};
        int maxpairs = 0;
        for (int i = 0; i < P.n_dirs; ++i) maxpairs = std::max(maxpairs, n3[P.dirs[i]] * (int)R);
        group[e] = std::min(512, (maxpairs + 63) / 64 * 64);  // the kernel is built for <= 512 threads
        c->con_block = std::max(c->con_block, group[e]);
    }
    c->con_lds = 0;
    for (int e = 0; e < n; ++e) {
        EnsDesc& E = c->h_ens[e];
        const int n3[3] = {E.nx, E.ny, E.nz};
        const size_t nmax = (size_t)std::max(E.nx, std::max(E.ny, E.nz));
        const size_t per = P.multihit ? 32 : 16;  // LDS bytes per (measurement, line site)
        E.con_lpb = c->con_block / group[e];
        const size_t fit = (size_t)kConLds / ((size_t)E.con_lpb * nmax * per);
        E.con_mc = (int)std::max<size_t>(1, std::min<size_t>(fit, (size_t)P.n_i));
        c->con_lds = std::max(c->con_lds, (size_t)E.con_lpb * E.con_mc * nmax * per);
        {
            const int len0 = n3[P.dirs[0]];
            bool same = e == 0 || c->ins_line_len == len0;
            for (int i = 0; i < P.n_dirs; ++i) same = same && n3[P.dirs[i]] == len0;
            c->ins_line_len = same ? len0 : 0;
        }
        if (!P.probes.empty() && !P.spectral && P.ins_ks == kMfSlots) {
            // matrix-core kernel: kMfThreads work-items, (slot block, y, 8
            // separations) tiles, up to 4 kMfTiles per pass over the
            // measurements; as many slot blocks per work-group as one pass
            // holds, fewer while a chunk would hold fewer than 8 measurements;
            // chunks of a multiple of 4 measurements
            const int nsb = (int)(P.pblk.size() / kInsBlkInts);
            const int unit = (int)(nmax * ((R + 7) / 8));
            const int cap = (kMfThreads / 64) * kMfTiles;
            E.ins_pbw = std::max(1, std::min(std::min(nsb, cap / std::max(1, unit)), kMfRows / (2 * kMfSlots)));
            auto fit_mc = [&](int bpw) {
                int mc = (std::min(P.n_i, kMfPh) + 3) / 4 * 4;
                while (mc > 4 && !mf_chunk_fits(mc, (int)nmax, (int)R, bpw * 2 * kMfSlots, (int)word)) mc -= 4;
                return mc;
            };
            while (E.ins_pbw > 1 && (!mf_chunk_fits(4, (int)nmax, (int)R, E.ins_pbw * 2 * kMfSlots, (int)word) ||
                                     fit_mc(E.ins_pbw) < std::min(8, (P.n_i + 3) / 4 * 4)))
                --E.ins_pbw;
            const int mc = fit_mc(E.ins_pbw);
            if (!mf_chunk_fits(mc, (int)nmax, (int)R, E.ins_pbw * 2 * kMfSlots, (int)word)) {
                release(c);
                return set_err(nullptr, U1ML_ENOTSUP, "history-form insertions: matrix-core chunk does not fit LDS");
            }
            c->ins_block = kMfThreads;
            E.ins_mc = mc;
        } else if (!P.probes.empty() && !P.spectral) {
            const int nsb = (int)(P.pblk.size() / kInsBlkInts);
            const int ks = P.ins_ks, kr = ins_kr(ks);
            const int unit = (int)(nmax * ((R + kr - 1) / kr));  // tasks of one slot block
            E.ins_pbw = std::max(1, std::min(std::min(nsb, kInsThreads / unit), kInsRowsMax / (2 * ks)));
            // ins_mc measurements per LDS chunk buffer (static LDS of the kernel):
            // fewer slot blocks per work-group while a chunk would hold fewer than 8
            auto fit_mc = [&](int bpw) {
                int mc = std::min(P.n_i, kInsPh);
                while (mc > 1 && !ins_chunk_fits(mc, (int)nmax, bpw * ks * 2, (int)word)) --mc;
                return mc;
            };
            // (fewer also while not even one measurement fits)
            while (E.ins_pbw > 1 && (!ins_chunk_fits(1, (int)nmax, E.ins_pbw * ks * 2, (int)word) ||
                                     fit_mc(E.ins_pbw) < std::min(8, P.n_i)))
                --E.ins_pbw;
            c->ins_block = std::max(c->ins_block, std::min(kInsThreads, (E.ins_pbw * unit + 63) / 64 * 64));
            const int nrows = E.ins_pbw * ks * 2;
            const int mc = fit_mc(E.ins_pbw);
            if (!ins_chunk_fits(mc, (int)nmax, nrows, (int)word)) {
                release(c);
                return set_err(nullptr, U1ML_ENOTSUP,
                               "history-form insertions: one measurement of a work-group's phases or O rows exceeds "
                               "its LDS buffer (use the spectral form)");
            }
            E.ins_mc = mc;
        }
        E.prod_nch = (P.n_dirs * E.nsig + kProdChunk - 1) / kProdChunk;
        E.res_index = e;
        long long n12max = 0;
        for (int i = 0; i < P.n_dirs; ++i) n12max = std::max<long long>(n12max, E.nsig / n3[P.dirs[i]]);
        c->spec_npm = std::max(c->spec_npm, std::max(E.nx, std::max(E.ny, E.nz)));
        c->spec_n12max = std::max(c->spec_n12max, n12max);
        for (int i = 0; i < P.n_dirs; ++i)
            for (int k = 1; k < 3; ++k)
                if (n3[(P.dirs[i] + k) % 3] % 4 != 0) c->spec_tile = 2;
    }
    // the whole batch as one lane; the split into lanes follows the streams below
    {
        Lane& L = c->whole;
        L.idx.resize(n);
        for (int e = 0; e < n; ++e) L.idx[e] = e;
        L.n = n;
        L.h_ens = c->h_ens;
        L.bmap_stride = Lo.bmap_stride;
        L.d_ens = (EnsDesc*)(s + Lo.s_ens);
        L.d_bstart = (int*)(s + Lo.s_bstart);
        L.d_bmap = (UpdBlock*)(s + Lo.s_bmap);
        L.d_mmap = (int2*)(s + Lo.s_mmap);
        L.d_ring = (int*)(s + Lo.s_ring);
        L.prodpart = (double*)(s + Lo.s_prodpart);
        L.stream = c->stream;
        build_lane_tables(c, L);
    }
    {
        // every dynamic LDS request must fit the device's limit per work-group
        int lds_max = 0;
        hipError_t ea = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
        const size_t plane_lds = P.spectral ? (2 * (size_t)c->spec_n12max + 2 * (size_t)c->spec_npm) * sizeof(double2) : 0;
        const size_t mac_lds = P.spectral ? spec_mac_lds(c->spec_npm) : 0;
        const size_t need = std::max(std::max(c->con_lds, c->ins_lds), std::max(plane_lds, mac_lds));
        if (ea != hipSuccess || (size_t)lds_max < need) {
            release(c);
            return set_err(nullptr, ea != hipSuccess ? U1ML_EDEVICE : U1ML_ENOTSUP,
                           "work-group LDS of " + std::to_string(need) + " bytes exceeds the device limit of " +
                               std::to_string(lds_max));
        }
    }
    std::vector<uint32_t> zeros(n, 0u);
    u1ml_status st = U1ML_OK;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (st != U1ML_OK || bytes == 0) return;
        hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) st = set_err(nullptr, U1ML_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    };
    up(c->d_obs, &O, sizeof O);
    up(c->d_r, P.r.data(), sizeof(int) * P.r.size());
    up(c->d_probe, probe_flat.data(), sizeof(int) * probe_flat.size());
    up(c->d_comp, P.comps.data(), sizeof(int) * P.comps.size());
    up(c->d_pgroup, P.pgroup.data(), sizeof(int) * P.pgroup.size());
    up(c->d_gdesc, P.gdesc.data(), sizeof(int) * P.gdesc.size());
    up(c->d_pblk, P.pblk.data(), sizeof(int) * P.pblk.size());
    up(c->d_upd, zeros.data(), sizeof(uint32_t) * n);
    if (st == U1ML_OK) {
        hipError_t e = upload_lane(c->whole);
        if (e != hipSuccess) st = set_err(nullptr, U1ML_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    if (st == U1ML_OK) {
        hipError_t e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
        for (int l = 1; l < kMaxLanes && e == hipSuccess; ++l) {
            e = hipStreamCreateWithFlags(&c->lane_stream[l], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join[l], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = split_lanes(c, std::min(n, default_lanes(P.precision)));
        if (e != hipSuccess) st = set_err(nullptr, U1ML_EDEVICE, std::string("lanes: ") + hipGetErrorString(e));
    }
    if (st != U1ML_OK) {
        release(c);
        return st;
    }
    *out = c;
    return U1ML_OK;
}

u1ml_status u1ml_destroy(u1ml_ctx* ctx)
{
    if (!ctx) return U1ML_OK;
    // every lane joins the context's stream, so this waits for all work that
    // still reads the workspace or runs the graphs about to be destroyed
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    release(ctx);
    return e == hipSuccess ? U1ML_OK : set_err(nullptr, U1ML_EDEVICE, std::string("u1ml_destroy: ") + hipGetErrorString(e));
}

u1ml_status u1ml_init_links(u1ml_ctx* ctx, int start)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (start != U1ML_COLD && start != U1ML_HOT) return set_err(ctx, U1ML_EINVAL, "start must be 0 (cold) or 1 (hot)");
    HIPCHK(ctx, launch_init_links(ctx->whole.d_ens, ctx->whole.tab_dev(kTabAll), ctx->P.n_ens, ctx->whole.tab_total(kTabAll),
                                  ctx->P.precision, ctx->links, start, ctx->stream));
    HIPCHK(ctx, launch_fill_zero(ctx->d_upd, align_up(sizeof(uint32_t) * ctx->P.n_ens), ctx->stream));
    ctx->initialised = true;
    return U1ML_OK;
}

u1ml_status u1ml_sweeps(u1ml_ctx* ctx, int n)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (n < 0) return set_err(ctx, U1ML_EINVAL, "n must be >= 0");
    if (!ctx->initialised) return set_err(ctx, U1ML_ESTATE, "links not initialised");
    if (n == 0) return U1ML_OK;
    // one lane's n sweeps on its stream (graph of one sweep, launched n times)
    auto lane_sweeps = [&](Lane& L) -> hipError_t {
        if (ctx->use_graphs) {
            if (!L.g_sweep &&
                capture(ctx, [&](hipStream_t st) { return enq_sweep_with_counter(ctx, L, st); }, &L.g_sweep) != U1ML_OK)
                return hipErrorUnknown;
            for (int i = 0; i < n; ++i) {
                hipError_t e = hipGraphLaunch(L.g_sweep, L.stream);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        for (int i = 0; i < n; ++i) {
            hipError_t e = enq_sweep_with_counter(ctx, L, L.stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const std::string before = ctx->err;
    hipError_t e = on_lanes(ctx, lane_sweeps);
    if (e != hipSuccess)
        return ctx->err != before && e == hipErrorUnknown ? U1ML_EDEVICE
                                                          : set_err(ctx, U1ML_EDEVICE, std::string("sweeps: ") + hipGetErrorString(e));
    return U1ML_OK;
}

u1ml_status u1ml_phase(u1ml_ctx* ctx, int kind, int mu, int parity, int tau, int pass_offset)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (!ctx->initialised) return set_err(ctx, U1ML_ESTATE, "links not initialised");
    if ((kind < 0 || kind > 2) || mu < 0 || mu > 3 || (parity != 0 && parity != 1) || pass_offset < 0)
        return set_err(ctx, U1ML_EINVAL, "bad phase arguments");
    bool ok;
    update_class(ctx, mu, tau, &ok);
    if (!ok) return set_err(ctx, U1ML_EINVAL, "tau must be <= 1 or one of the problem's level thicknesses");
    HIPCHK(ctx, enq_phase(ctx, ctx->whole, ctx->stream, kind, mu, parity, tau, pass_offset));
    return U1ML_OK;
}

u1ml_status u1ml_multilevel(u1ml_ctx* ctx)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (!ctx->initialised) return set_err(ctx, U1ML_ESTATE, "links not initialised");
    if (ctx->ring_count >= ctx->P.max_configs)
        return set_err(ctx, U1ML_ESTATE, "results ring is full: call u1ml_copy_results");
    const bool graph = ctx->use_graphs && body_launches(ctx->P) <= kMaxGraphLaunches;
    auto lane_config = [&](Lane& L) -> hipError_t {
        if (!graph) return enq_multilevel(ctx, L, L.stream);
        if (!L.g_ml && capture(ctx, [&](hipStream_t st) { return enq_multilevel(ctx, L, st); }, &L.g_ml) != U1ML_OK)
            return hipErrorUnknown;
        return hipGraphLaunch(L.g_ml, L.stream);
    };
    const std::string before = ctx->err;
    hipError_t e = on_lanes(ctx, lane_config);
    if (e != hipSuccess)
        return ctx->err != before && e == hipErrorUnknown
                   ? U1ML_EDEVICE
                   : set_err(ctx, U1ML_EDEVICE, std::string("multilevel: ") + hipGetErrorString(e));
    ctx->ring_count++;
    return U1ML_OK;
}

u1ml_status u1ml_copy_results(u1ml_ctx* ctx, double* host, size_t n_doubles, size_t* n_written)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (!host && n_doubles) return set_err(ctx, U1ML_EINVAL, "host is NULL");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const size_t avail = (size_t)ctx->ring_count * ctx->P.n_ens * (size_t)ctx->P.nd_cfg;
    const size_t nw = std::min(avail, n_doubles);
    if (nw) HIPCHK(ctx, hipMemcpy(host, ctx->res, nw * sizeof(double), hipMemcpyDeviceToHost));
    int zero[4] = {0, 0, 0, 0};
    for (Lane* L : all_lanes(ctx))
        if (L->n) HIPCHK(ctx, hipMemcpy(L->d_ring, zero, sizeof zero, hipMemcpyHostToDevice));
    ctx->ring_count = 0;
    if (n_written) *n_written = nw;
    return U1ML_OK;
}

u1ml_status u1ml_get_links(u1ml_ctx* ctx, int ens, double* host, size_t n)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (ens < 0 || ens >= ctx->P.n_ens) return set_err(ctx, U1ML_EINVAL, "ensemble index out of range");
    const long long V = 2ll * ctx->h_ens[ens].vh;
    if (!host || n != (size_t)(4 * V)) return set_err(ctx, U1ML_EINVAL, "host buffer must hold exactly 4 V doubles");
    HIPCHK(ctx, launch_gather_links(ctx->whole.d_ens, ens, ctx->P.precision, ctx->links, ctx->stage, V, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(host, ctx->stage, sizeof(double) * 4 * V, hipMemcpyDeviceToHost));
    return U1ML_OK;
}

u1ml_status u1ml_set_links(u1ml_ctx* ctx, int ens, const double* host, size_t n)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (ens < 0 || ens >= ctx->P.n_ens) return set_err(ctx, U1ML_EINVAL, "ensemble index out of range");
    const long long V = 2ll * ctx->h_ens[ens].vh;
    if (!host || n != (size_t)(4 * V)) return set_err(ctx, U1ML_EINVAL, "host buffer must hold exactly 4 V doubles");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(ctx->stage, host, sizeof(double) * 4 * V, hipMemcpyHostToDevice));
    HIPCHK(ctx, launch_scatter_links(ctx->whole.d_ens, ens, ctx->P.precision, ctx->links, ctx->stage, V, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->initialised = true;
    return U1ML_OK;
}

u1ml_status u1ml_get_counter(u1ml_ctx* ctx, int ens, uint32_t* counter)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (ens < 0 || ens >= ctx->P.n_ens || !counter) return set_err(ctx, U1ML_EINVAL, "bad arguments");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(counter, ctx->d_upd + ens, sizeof(uint32_t), hipMemcpyDeviceToHost));
    return U1ML_OK;
}

u1ml_status u1ml_set_counter(u1ml_ctx* ctx, int ens, uint32_t counter)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (ens < 0 || ens >= ctx->P.n_ens) return set_err(ctx, U1ML_EINVAL, "bad arguments");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(ctx->d_upd + ens, &counter, sizeof(uint32_t), hipMemcpyHostToDevice));
    return U1ML_OK;
}

u1ml_status u1ml_plaquette(u1ml_ctx* ctx, double* out)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (!out) return set_err(ctx, U1ML_EINVAL, "out is NULL");
    if (!ctx->initialised) return set_err(ctx, U1ML_ESTATE, "links not initialised");
    HIPCHK(ctx, launch_plaquette(ctx->whole.d_ens, ctx->P.n_ens, 0, ctx->P.precision, ctx->links, ctx->ppart, ctx->pout,
                                 ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(out, ctx->pout, sizeof(double) * 6 * ctx->P.n_ens, hipMemcpyDeviceToHost));
    return U1ML_OK;
}

u1ml_status u1ml_plaquette_noalloc(u1ml_ctx* ctx, double* d_out)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (!d_out) return set_err(ctx, U1ML_EINVAL, "d_out is NULL");
    if (ctx->P.n_ens > kStaticPlaqEns)
        return set_err(ctx, U1ML_EINVAL,
                       "u1ml_plaquette_noalloc takes at most " + std::to_string(kStaticPlaqEns) + " ensembles");
    if (!ctx->initialised) return set_err(ctx, U1ML_ESTATE, "links not initialised");
    HIPCHK(ctx, launch_plaquette(ctx->whole.d_ens, ctx->P.n_ens, 0, ctx->P.precision, ctx->links,
                                 ctx->static_partials, d_out, ctx->stream));
    return U1ML_OK;
}

u1ml_status u1ml_health(u1ml_ctx* ctx, uint64_t* n_bad)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (!n_bad) return set_err(ctx, U1ML_EINVAL, "n_bad is NULL");
    HIPCHK(ctx, launch_fill_zero(ctx->d_count, 16, ctx->stream));
    HIPCHK(ctx, launch_health(ctx->whole.d_ens, ctx->whole.tab_dev(kTabAll), ctx->P.n_ens, ctx->whole.tab_total(kTabAll),
                              ctx->P.precision, ctx->links, ctx->d_count, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    unsigned long long v = 0;
    HIPCHK(ctx, hipMemcpy(&v, ctx->d_count, sizeof v, hipMemcpyDeviceToHost));
    *n_bad = v;
    return U1ML_OK;
}

u1ml_status u1ml_set_block(u1ml_ctx* ctx, int block)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
        return set_err(ctx, U1ML_EINVAL, "block must be 64, 128, 256, 512 or 1024");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->block = block;
    for (Lane* L : all_lanes(ctx)) {
        if (!L->n) continue;
        build_update_tabs(ctx, *L);
        HIPCHK(ctx, hipMemcpy(L->d_bstart, L->h_bstart.data(), sizeof(int) * 4 * (L->n + 1), hipMemcpyHostToDevice));
        HIPCHK(ctx, hipMemcpy(L->d_bmap, L->h_bmap.data(), sizeof(UpdBlock) * L->h_bmap.size(), hipMemcpyHostToDevice));
    }
    drop_graphs(ctx);
    return U1ML_OK;
}

u1ml_status u1ml_set_lanes(u1ml_ctx* ctx, int n_lanes)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (n_lanes < 1 || n_lanes > kMaxLanes) return set_err(ctx, U1ML_EINVAL, "n_lanes must be 1, 2, 3 or 4");
    if (n_lanes > ctx->P.n_ens) return set_err(ctx, U1ML_EINVAL, "more lanes than ensembles");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (n_lanes != ctx->n_lanes) HIPCHK(ctx, split_lanes(ctx, n_lanes));
    // the lanes now in use continue the results ring where it stands
    const int ring[4] = {ctx->ring_count, 0, 0, 0};
    for (Lane* L : all_lanes(ctx))
        if (L->n) HIPCHK(ctx, hipMemcpy(L->d_ring, ring, sizeof ring, hipMemcpyHostToDevice));
    return U1ML_OK;
}

u1ml_status u1ml_set_graphs(u1ml_ctx* ctx, int enable)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    ctx->use_graphs = enable != 0;
    return U1ML_OK;
}

namespace {
// Average device time of n_rep launches of one phase by lane L on the
// context's stream, each launch with its own start/stop event pair.
u1ml_status time_lane_phase(u1ml_ctx* ctx, const Lane& L, int kind, int mu, int parity, int tau, int n_rep, double* us)
{
    if (!us || n_rep < 1 || kind < 0 || kind > 2 || mu < 0 || mu > 3 || (parity & ~1))
        return set_err(ctx, U1ML_EINVAL, "bad arguments");
    if (!ctx->initialised) return set_err(ctx, U1ML_ESTATE, "links not initialised");
    bool ok;
    update_class(ctx, mu, tau, &ok);
    if (!ok) return set_err(ctx, U1ML_EINVAL, "tau must be <= 1 or one of the problem's level thicknesses");
    // every launch carries its own start/stop events, which take the dispatch's
    // begin and end timestamps: the average is the kernel's own duration, the
    // figure a kernel trace reports, without the launch gaps between dispatches
    std::vector<hipEvent_t> ev(2 * (size_t)n_rep, nullptr);
    for (auto& x : ev) HIPCHK(ctx, hipEventCreate(&x));
    hipError_t he = hipSuccess;
    for (int i = 0; i < n_rep && he == hipSuccess; ++i)
        he = enq_phase(ctx, L, ctx->stream, kind, mu, parity, tau, 0, ev[2 * i], ev[2 * i + 1]);
    if (he == hipSuccess) he = hipEventSynchronize(ev.back());
    double total = 0.0;
    for (int i = 0; i < n_rep && he == hipSuccess; ++i) {
        float ms = 0.f;
        he = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
        total += ms;
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (he != hipSuccess) return set_err(ctx, U1ML_EDEVICE, std::string("time_phase: ") + hipGetErrorString(he));
    *us = 1000.0 * total / n_rep;
    return U1ML_OK;
}
}  // namespace

u1ml_status u1ml_time_phase(u1ml_ctx* ctx, int kind, int mu, int parity, int tau, int n_rep, double* us)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    return time_lane_phase(ctx, ctx->whole, kind, mu, parity, tau, n_rep, us);
}

u1ml_status u1ml_time_phase_lane(u1ml_ctx* ctx, int lane, int kind, int mu, int parity, int tau, int n_rep,
                                 double* us, double* bytes, long* updates)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (lane < 0 || lane >= ctx->n_lanes) return set_err(ctx, U1ML_EINVAL, "lane out of range");
    if (!bytes || !updates) return set_err(ctx, U1ML_EINVAL, "bad arguments");
    const Lane& L = ctx->n_lanes <= 1 ? ctx->whole : ctx->split[lane];
    const u1ml_status st = time_lane_phase(ctx, L, kind, mu, parity, tau, n_rep, us);
    if (st != U1ML_OK) return st;
    const double word = ctx->P.precision == U1ML_FP64 ? 8.0 : 4.0;
    double b = 0;
    long u = 0;
    for (int e : L.idx) {
        long long w, uu;
        phase_words(ctx->P.ens[e], kind, mu, parity, tau, &w, &uu);
        b += w * word;
        u += (long)uu;
    }
    *bytes = b;
    *updates = u;
    return U1ML_OK;
}

u1ml_status u1ml_phase_bytes(u1ml_ctx* ctx, int kind, int mu, int parity, int tau, double* bytes, long* updates)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (!bytes || !updates || mu < 0 || mu > 3 || (parity & ~1) || kind < 0 || kind > 2)
        return set_err(ctx, U1ML_EINVAL, "bad arguments");
    const double word = ctx->P.precision == U1ML_FP64 ? 8.0 : 4.0;
    double b = 0;
    long u = 0;
    for (const u1ml_ensemble& E : ctx->P.ens) {
        long long w, uu;
        phase_words(E, kind, mu, parity, tau, &w, &uu);
        b += w * word;
        u += (long)uu;
    }
    *bytes = b;
    *updates = u;
    return U1ML_OK;
}

u1ml_status u1ml_autotune(u1ml_ctx* ctx, u1ml_tune_report* report)
{
    if (!ctx) return set_err(nullptr, U1ML_EINVAL, "ctx is NULL");
    if (!ctx->initialised) return set_err(ctx, U1ML_ESTATE, "links not initialised");
    const int cand[5] = {64, 128, 256, 512, 1024};
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    // save links and counters so tuning leaves no trace
    const size_t lbytes = ctx->Lo.sz_links;
    void* saved = nullptr;
    HIPCHK(ctx, hipMalloc(&saved, lbytes));
    hipError_t he = hipMemcpy(saved, ctx->links, lbytes, hipMemcpyDeviceToDevice);
    std::vector<uint32_t> upd(ctx->P.n_ens);
    if (he == hipSuccess) he = hipMemcpy(upd.data(), ctx->d_upd, sizeof(uint32_t) * upd.size(), hipMemcpyDeviceToHost);
    if (he != hipSuccess) {
        (void)hipFree(saved);
        return set_err(ctx, U1ML_EDEVICE, std::string("autotune save: ") + hipGetErrorString(he));
    }
    const int old_block = ctx->block;
    const bool old_graphs = ctx->use_graphs;
    ctx->use_graphs = false;
    double best = 1e300;
    int best_b = old_block;
    u1ml_tune_report rep;
    std::memset(&rep, 0, sizeof rep);
    u1ml_status st = U1ML_OK;
    const int tau = ctx->P.tau_i;
    for (int i = 0; i < 5 && st == U1ML_OK; ++i) {
        st = u1ml_set_block(ctx, cand[i]);
        if (st != U1ML_OK) break;
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            st = set_err(ctx, U1ML_EDEVICE, "event creation failed");
            break;
        }
        hipError_t e = enq_sweep(ctx, ctx->whole, ctx->stream, tau, 0);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(a, ctx->stream);
        for (int k = 0; k < 5 && e == hipSuccess; ++k) e = enq_sweep(ctx, ctx->whole, ctx->stream, tau, 0);
        if (e == hipSuccess) e = hipEventRecord(b, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (e != hipSuccess) {
            st = set_err(ctx, U1ML_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
            break;
        }
        rep.block[i] = cand[i];
        rep.us_per_sweep[i] = 1000.0 * ms / 5;
        rep.n_candidates = i + 1;
        if (rep.us_per_sweep[i] < best) {
            best = rep.us_per_sweep[i];
            best_b = cand[i];
        }
    }
    hipError_t e1 = hipMemcpy(ctx->links, saved, lbytes, hipMemcpyDeviceToDevice);
    hipError_t e2 = hipMemcpy(ctx->d_upd, upd.data(), sizeof(uint32_t) * upd.size(), hipMemcpyHostToDevice);
    (void)hipFree(saved);
    ctx->use_graphs = old_graphs;
    if (st != U1ML_OK) {
        u1ml_set_block(ctx, old_block);
        return st;
    }
    if (e1 != hipSuccess || e2 != hipSuccess) return set_err(ctx, U1ML_EDEVICE, "autotune restore failed");
    st = u1ml_set_block(ctx, best_b);
    rep.chosen_block = best_b;
    if (report) *report = rep;
    return st;
}

u1ml_status u1ml_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, size_t n,
                             uint32_t* d_out, void* hip_stream)
{
    if (!d_out && n) return set_err(nullptr, U1ML_EINVAL, "d_out is NULL");
    if (n > 0xFFFFFFFFull) return set_err(nullptr, U1ML_EINVAL, "n must be < 2^32");
    hipError_t e = launch_philox_fill(k0, k1, c0, c1, c2, c3, n, d_out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return set_err(nullptr, U1ML_EDEVICE, hipGetErrorString(e));
    return U1ML_OK;
}

u1ml_status u1ml_sincos_fill(const double* d_x, size_t n, double* d_s, double* d_c, void* hip_stream)
{
    if ((!d_x || !d_s || !d_c) && n) return set_err(nullptr, U1ML_EINVAL, "NULL device pointer");
    if (n > 0xFFFFFFFFull) return set_err(nullptr, U1ML_EINVAL, "n must be < 2^32");
    hipError_t e = launch_sincos_fill(d_x, n, d_s, d_c, (hipStream_t)hip_stream);
    if (e != hipSuccess) return set_err(nullptr, U1ML_EDEVICE, hipGetErrorString(e));
    return U1ML_OK;
}

u1ml_status u1ml_vonmises_fill(double kappa, int precision, uint32_t seed, uint32_t key_id, uint32_t c0, uint32_t c1,
                               size_t n, double* d_out, int* d_attempts, void* hip_stream)
{
    if (!d_out && n) return set_err(nullptr, U1ML_EINVAL, "d_out is NULL");
    if (!(kappa >= 0) || !std::isfinite(kappa)) return set_err(nullptr, U1ML_EINVAL, "kappa must be finite and >= 0");
    if (precision != U1ML_FP64 && precision != U1ML_FP32) return set_err(nullptr, U1ML_EINVAL, "bad precision");
    if (n > 0xFFFFFFFFull) return set_err(nullptr, U1ML_EINVAL, "n must be < 2^32");
    hipError_t e = launch_vonmises_fill(kappa, precision, seed, key_id, c0, c1, n, d_out, d_attempts,
                                        (hipStream_t)hip_stream);
    if (e != hipSuccess) return set_err(nullptr, U1ML_EDEVICE, hipGetErrorString(e));
    return U1ML_OK;
}

}  // extern "C"
