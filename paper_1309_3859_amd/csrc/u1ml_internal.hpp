// u1ml_internal.hpp -- data shared by the host scheduler and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace u1ml {

// Per-ensemble descriptor, resident in device memory.  Offsets are element
// offsets into the workspace sections (links: real; history phases, slab
// averages and outer sums: double2; history O sums: double).
struct EnsDesc {
    int nx, ny, nz, nt;
    int nxh, nsig, vh, s_in;  // s_in: slabs of the innermost level
    int s_out, n_vac_blocks;
    int con_lpb, con_mc;  // contraction: lines per work-group, measurements per LDS chunk
    int prod_nch;   // slab products: site chunks per (r, probe)
    int res_index;  // index of the ensemble in the problem (counters, results)
    int ins_pbw, ins_mc;  // insertion contraction: slot blocks per work-group, measurements per LDS chunk
    float inv_nxh, inv_ny, inv_slice, pad3;  // 1/(Nx/2), 1/Ny, 1/((Nx/2) Ny Nz) for division-free decode
    double beta, sqrt_beta;
    double metro_delta;  // Metropolis proposal step
    uint32_t seed, key_id;
    long long link_off;
    long long hc_off, ho_off;
    long long hcm_off;  // multihit slab phases (double2), [m][s][site], when multihit
    long long at_off, ato_off;
    long long ot_off, oto_off;
    long long vac_part_off;  // double, [n_vac_blocks][12][hi, lo]: running sums over the configuration's measurements
    // spectral form (double2 offsets)
    long long wf_off, gf_off, sph_off, spo_off, facc_off;
    long long cpl_off, opl_off;  // plane-major copies of one measurement's slab phases (double2) and O rows (real)
};

// One work-group of an update launch: its ensemble and block index within it
// (a padding block of the XCD-aware order has an index past the ensemble's
// links), the number of links of the ensemble that the launch's phase class
// updates, and the geometry the update kernel needs before its loads, so that
// one 64-byte scalar load replaces a block-map load followed by descriptor
// loads.
struct alignas(64) UpdBlock {
    int e, blk;
    int nx, ny, nz, nt, nxh, vh;
    float inv_slice, inv_nxh, inv_ny;
    int res_index;
    long long link_off;
    int n_items;  // non-frozen links of one (direction, parity) of this class
    int pad1;
};
static_assert(sizeof(UpdBlock) == 64, "UpdBlock is one 64-byte scalar load");

// Observable tables in device memory.
struct ObsDesc {
    int n_dirs;
    int dirs[3];
    int n_r, n_probe, n_comp;
    int store_o;  // 1 if insertions are requested (history keeps O sums)
    int n_groups;  // probe groups sharing (l, mode) (spectral form)
    int n_ens_total;  // ensembles of the problem (rows of a results record)
    int multihit;     // correlator averages from multihit slab phases
    int n_pblocks;    // insertion contraction: slot blocks (probe, component pairs sharing (l, mode, spans))
    long long n_doubles_per_config;
};

// Insertion contraction (history form): the (probe, component) slots that
// share (l, mode, spans) meet every T value at the same offset along the axis
// and form blocks of KS slots (9, 6, 3 or 1, the planner's choice); a
// work-item owns one position y of the displaced lines, ins_kr(KS)
// separations and one slot block (KR x KS x 4 FP64 accumulators).  A slot
// block is kInsBlkInts ints: l, mode, spans (0 or 1), number of slots, then
// per slot its probe index, component index (into the problem's list), p1, p2.
constexpr int kInsSlotMax = 9;
constexpr int kInsBlkInts = 4 + 4 * kInsSlotMax;
constexpr int kInsThreads = 256;  // largest work-group
constexpr int kInsPh = 384;       // phases of one LDS chunk buffer (16-byte vectors, a multiple of 64)
constexpr int kInsOb = 25600;     // O rows of one LDS chunk buffer (bytes, a multiple of 1024)
constexpr int kInsRowsMax = 512;  // O rows (slot block, slot, kind) of one work-group
__host__ __device__ constexpr int ins_kr(int ks) { return ks == 9 ? 2 : (ks == 6 ? 3 : (ks == 3 ? 4 : 8)); }
// measurements per chunk buffer of the contraction: the phases [q][x] and the
// O rows [q][row][y] (word bytes each) of mc measurements, each region
// rounded up to whole waves of 64 16-byte vectors, must fit kInsPh and kInsOb
__host__ __device__ inline bool ins_chunk_fits(int mc, int N, int nrows, int word)
{
    const size_t ph = ((size_t)mc * N + 63) / 64 * 64;
    const size_t ob = ((size_t)mc * nrows * N * word + 1023) / 1024 * 1024;
    return ph <= (size_t)kInsPh && ob <= (size_t)kInsOb;
}

// The same sums on the matrix cores: for one position y of a slot block the
// sums over measurements are a product of a (separation, re/im) x measurement
// matrix of T values and a measurement x (slot, kind) matrix of O values, one
// 16 x 16 FP64 tile per 8 separations and 8 slots, 4 measurements per MFMA
// step.  Slot blocks of kMfSlots; a work-group of kMfThreads work-items keeps
// kMfTiles tiles per wave; per chunk of measurements the LDS holds the line's
// phases and O rows (copied straight from memory, double-buffered) and the T
// values of every (measurement, x, separation) computed once from the phases.
constexpr int kMfSlots = 8;
constexpr int kMfThreads = 256;
constexpr int kMfTiles = 12;   // accumulator tiles per wave (4 FP64 each per work-item)
constexpr int kMfPh = 256;     // phases of one chunk buffer (16-byte vectors)
constexpr int kMfOb = 16384;   // O rows of one chunk buffer (bytes)
constexpr int kMfT = 4608;     // T values of a chunk (doubles)
constexpr int kMfRows = 256;   // O rows (slot block, slot, kind) of one work-group
constexpr int kMfR = 64;       // separations
// O rows in LDS: [q][row][y] with a row stride of at most the row's words
// plus 4 (16-byte copies; else one element more than the row, an odd
// stride whose reads at one y fall in distinct banks)
__host__ __device__ inline int mf_row_dwords(int N, int word) { return N * (word / 4) + 4; }
__host__ __device__ inline bool mf_chunk_fits(int mc, int N, int R, int nrows, int word)
{
    return (size_t)mc * N <= (size_t)kMfPh && (size_t)mc * nrows * mf_row_dwords(N, word) * 4 <= (size_t)kMfOb &&
           (size_t)mc * N * 2 * R <= (size_t)kMfT && nrows <= kMfRows && R <= kMfR;
}

constexpr int kUpdateClasses = 4;  // temporal, spatial full, spatial inner tau, spatial outer tau
constexpr int kProdChunk = 2048;    // slab products: (axis, site) items per work-group
constexpr int kProdQ = 26;          // slab products: correlator re, im and 12 insertion quantities re, im
constexpr int kConLds = 49152;      // contraction: LDS budget per work-group (bytes)
constexpr int kPlaqBlocks = 1024;   // plaquette means: work-groups (and partials) per ensemble
constexpr int kStaticPlaqEns = 32;  // allocation-free plaquettes: ensembles whose partials fit the static scratch

// --- launchers (k_update.hip) ---
hipError_t launch_init_links(const EnsDesc* d_ens, const int* d_bstart_all, int n_ens, int total_blocks, int precision,
                             void* links, int start, hipStream_t st);
// d_blocks[b]: ensemble, block index within the ensemble and geometry of every block of the launch;
// ev_start/ev_stop (both or neither) record the dispatch's begin and end timestamps
hipError_t launch_update(const EnsDesc* d_ens, const UpdBlock* d_blocks, int total_blocks, int block, int precision,
                         void* links, const uint32_t* d_upd, int pass_offset, int kind, int mu, int parity, int tau,
                         hipStream_t st, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
hipError_t launch_health(const EnsDesc* d_ens, const int* d_bstart_all, int n_ens, int total_blocks, int precision,
                         const void* links, unsigned long long* d_count, hipStream_t st);
hipError_t launch_plaquette(const EnsDesc* d_ens, int n_ens, int max_blocks_per_ens, int precision, const void* links,
                            double* d_partials, double* d_out, hipStream_t st);
// device address, on the current device, of the library's static scratch of
// kStaticPlaqEns * kPlaqBlocks * 6 doubles (resolved once per device)
hipError_t static_scratch(double** ptr);
hipError_t launch_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, size_t n,
                              uint32_t* d_out, hipStream_t st);
hipError_t launch_vonmises_fill(double kappa, int precision, uint32_t seed, uint32_t key_id, uint32_t c0, uint32_t c1,
                                size_t n, double* d_out, int* d_att, hipStream_t st);
hipError_t launch_sincos_fill(const double* d_x, size_t n, double* d_s, double* d_c, hipStream_t st);
hipError_t launch_advance_counters(const EnsDesc* d_ens, uint32_t* d_upd, int n_ens, int delta, hipStream_t st);
hipError_t launch_gather_links(const EnsDesc* d_ens, int ens, int precision, const void* links, double* d_canon,
                               long long n_sites, hipStream_t st);
hipError_t launch_scatter_links(const EnsDesc* d_ens, int ens, int precision, void* links, const double* d_canon,
                                long long n_sites, hipStream_t st);

// --- launchers (k_measure.hip) ---
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_measure(const EnsDesc* d_ens, const int2* d_bmap, int total_blocks, int precision, const void* links,
                          double2* hist_c, void* hist_o, double* vac_part, int m_in, int m, int tau, int store_o,
                          int multihit, hipStream_t st);
// work-groups of `block` threads, each holding E.con_lpb lines; lds_bytes of dynamic LDS
hipError_t launch_contract(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, int block,
                           size_t lds_bytes, const ObsDesc* d_obs, const int* d_r, const double2* hist_c,
                           double2* avg_t, int n_meas, int max_slabs, int n_dirs, hipStream_t st);
// insertion averages [TO] of the inner level from the stored measurements
// work-groups of `block` threads; slots_per_block selects the kernel's tile (KS, ins_kr(KS)),
// kMfSlots the matrix-core kernel; line_len: the sites of every line of the launch where they
// are all the same (24 selects a build with constant LDS offsets), else 0
hipError_t launch_contract_ins(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, int block,
                               size_t lds_bytes, const ObsDesc* d_obs, const int* d_r, const int* d_comp,
                               const int* d_sblk, int slots_per_block, const double2* hist_c, const void* hist_o,
                               double2* avg_to, int n_meas, int precision, int max_slabs, int n_dirs, int line_len,
                               hipStream_t st);
hipError_t launch_combine(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, const ObsDesc* d_obs,
                          const double2* avg_t, const double2* avg_to, double2* out_t, double2* out_to, int q,
                          hipStream_t st);
// Slab products relative to 2^E(r), E(r) the largest binary exponent of the per-site correlator
// products; launch_prod_exp finds E(r) and writes it to the current record (where launch_product,
// launch_wfac and launch_gfac read it); launch_product runs it first.
// d_bstart: per ensemble n_r * n_pgroups * E.prod_nch work-groups; part: 52 doubles per work-group
hipError_t launch_prod_exp(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks,
                           const ObsDesc* d_obs, int n_r, int n_pgroups, const double2* src_t, int use_outer,
                           double scale, double* part, double* results, const int* d_ring, hipStream_t st);
hipError_t launch_product(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks,
                          const ObsDesc* d_obs, int n_r, int n_pgroups, const double2* src_t, const double2* src_to,
                          int use_outer, double scale, double* part, double* results, const int* d_ring,
                          hipStream_t st);
hipError_t launch_vac_final(const EnsDesc* d_ens, int n_ens, const ObsDesc* d_obs, const double* vac_part,
                            int n_meas, double* results, const int* d_ring, hipStream_t st);
hipError_t launch_ring_advance(int* d_ring, hipStream_t st);

// --- spectral form (k_spectral.hip) ---
// weights relative to 2^E(r) (read from the current record; gfac only when wf is null)
hipError_t launch_wfac(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, const ObsDesc* d_obs,
                       const double2* out_t, double scale, double2* wf, const double* results, const int* d_ring,
                       hipStream_t st);
hipError_t launch_gfac(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, const ObsDesc* d_obs,
                       const double2* avg_t, const double2* wf, int q, double2* gf, const double* results,
                       const int* d_ring, hipStream_t st);
// measurement m_in's slab phases and O rows copied to the plane-major order of each charge axis;
// d_bstart: per ensemble n_dirs * s_in * ceil(Nx/32) * ceil(max extent/32) * max extent work-groups
hipError_t launch_plane_stage(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks,
                              const ObsDesc* d_obs, const double2* hist_c, const void* hist_o, int m_in,
                              int precision, double2* cpl, void* opl, hipStream_t st);
hipError_t launch_dft_planes(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, size_t lds_bytes,
                             const ObsDesc* d_obs, const int* d_r, const double2* cpl, const void* opl,
                             const double2* gf, double2* sph, double2* spo, int precision, int tile,
                             hipStream_t st);
// spectral sums: work-groups of kMacThreads per (axis, slab, probe group, kMacK values of k);
// dynamic LDS spec_mac_lds(largest extent)
constexpr int kMacK = 8;
constexpr int kMacThreads = 192;
constexpr int kMacComps = 6;
inline size_t spec_mac_lds(int npm) { return (size_t)12 * npm * kMacK * 16; }
hipError_t launch_spec_mac(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, int npm,
                           const ObsDesc* d_obs, const int* d_r, const int* d_comp, const int* d_gdesc,
                           const double2* sph, const double2* spo, double2* facc, hipStream_t st);
hipError_t launch_spec_final(const EnsDesc* d_ens, int n_ens, const ObsDesc* d_obs, long long n_outputs, int npm,
                             const int* d_probe, const int* d_pgroup, const double2* facc, double n_meas_total,
                             double* results, const int* d_ring, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st);

}  // namespace u1ml
