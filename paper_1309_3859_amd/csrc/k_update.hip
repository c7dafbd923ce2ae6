// k_update.hip -- link initialisation and the checkerboard link update.
//
// Paper: Amado, Cardoso, Bicudo, arXiv 1309.3859, Sec. II (Wilson action,
// local updates with 3 overrelaxation steps), Sec. II.C.1 and Algorithm 1
// (sublattice updates with frozen boundary spatial links), Sec. II.D (links
// as phases, even then odd sites, in place).
//
// One work-item per link of the phase (direction mu, parity p, not frozen),
// every ensemble of the batch in the same launch: work-group b reads its
// ensemble, its block index within that ensemble and the geometry from one
// record (UpdBlock), the records dealt to the 8 XCDs in contiguous stretches
// and, within an ensemble, ordered time slice fastest (set by the host).
// The staple of a link reads 18 angles: 12 of the other parity (coalesced,
// shifted by one site), 6 of the same parity; none of them is written by the
// phase, so the update is in place.  The all-link kernels below (start,
// health check, canonical gather and scatter, plaquettes) find their ensemble
// from block start offsets or a fixed number of blocks per ensemble.
#include "device_common.hpp"
#include <hip/hip_ext.h>

#include <mutex>

#include "u1ml_internal.hpp"

namespace u1ml {

__device__ inline int find_ens(const int* __restrict__ bstart, int n_ens, int bid)
{
    int e = 0;
    while (e + 1 < n_ens && bid >= bstart[e + 1]) ++e;
    return e;
}

template <typename real>
struct LinkView {
    const real* base;
    int vh, nxh, ny, nz;
    __device__ inline real ld(int dir, int par, Coord c) const
    {
        const int h = (c.x >> 1) + nxh * (c.y + ny * (c.z + nz * c.t));
        return base[(size_t)(dir * 2 + par) * vh + h];
    }
};

// kind 0: heatbath theta = wrap(psi - arg A), psi ~ vonMises(0, beta |A|);
// kind 1: overrelaxation theta = wrap(-theta - 2 arg A) (unchanged if A = 0);
// kind 2: Metropolis (the paper's update), one hit per link.
// Staple sum A = sum_{nu != mu} exp(i phi_f) + exp(i phi_b), nu ascending,
// forward before backward, phi_f = v0 - v1 - v2, phi_b = v3 - v4 - v5.
//
// Heatbath: every lane makes the first two rejection attempts (one Philox
// block); the links still pending (about 1 in 10) are compacted, in lane
// order, into a queue in LDS and finished by consecutive threads, so a wave no
// longer waits for its slowest lane.  A link's result depends only on its own
// counters, so the queue changes no result.  A queue entry holds what the
// link's final angle needs besides its deviate: the staple sum A, theta =
// arg(e^{i psi} conj A) by one atan2 (wrap(psi - arg A) up to rounding).
template <typename real>
struct RetryQ;
template <>
struct RetryQ<float> {
    float kappa, ar, ai;
    unsigned lid, off;
};
template <>
struct RetryQ<double> {
    double kappa, ar, ai;
    unsigned lid, off;
};

// the link's new angle from an accepted deviate
__device__ inline float hb_angle(const RetryQ<float>& q, float cp, float sp)
{
    const float th = atan2_fast(sp * q.ar - cp * q.ai, cp * q.ar + sp * q.ai);
    return th >= 3.14159265f ? -3.14159265f : th;
}
// FP64: e^{i theta} = e^{i psi} conj(A) / |A| with e^{i psi} = f + i sin psi,
// sin psi = +-sqrt((1 - f)(1 + f)) (1 - f and 1 + f exact where they
// cancel), so one atan2 gives theta = psi - arg A in [-pi, pi)
__device__ inline double hb_angle(const RetryQ<double>& q, double cp, double sp)
{
    const double th = M<double>::atan2_(sp * q.ar - cp * q.ai, cp * q.ar + sp * q.ai);
    return th >= M<double>::pi ? -M<double>::pi : th;
}

// attempts of one Philox block; true with the new angle if one accepted
__device__ inline bool hb_block(const RetryQ<float>& q, const BfEnvF32& v, const Block4& b, float* th)
{
    float cp, sp;
    if (!bf_pair_f32(v, b, &cp, &sp)) return false;
    *th = hb_angle(q, cp, sp);
    return true;
}
__device__ inline bool hb_block(const RetryQ<double>& q, double r, const Block4& b, double* th)
{
    double f;
    bool neg;
    if (!bf_pair_f64(q.kappa, r, b, &f, &neg)) return false;
    const double sp = M<double>::sqrt_((1.0 - f) * (1.0 + f));
    *th = hb_angle(q, f, neg ? -sp : sp);
    return true;
}
__device__ inline BfEnvF32 hb_env(const RetryQ<float>& q) { return bf_env_f32(q.kappa); }
__device__ inline double hb_env(const RetryQ<double>& q) { return bf_r_f64(q.kappa); }

template <typename real, int KIND, int MU>
__global__ void __launch_bounds__(1024) k_update(const EnsDesc* __restrict__ ens, const UpdBlock* __restrict__ blocks,
                                                 real* __restrict__ links, const uint32_t* __restrict__ upd,
                                                 int pass_offset, int parity, int tau, float inv_tm1)
{
    constexpr bool kQueue = KIND == 0;
    // a padding block of the XCD-aware order carries a block index past its
    // ensemble's links, so all its work-items are inactive (no branch on the
    // record, whose fields then all load at once)
    const UpdBlock B = blocks[blockIdx.x];
    const EnsDesc& E = ens[B.e];  // coupling, key and step: read after the link loads are issued
    const Geo g{B.nx, B.ny, B.nz, B.nt, B.nxh, B.nxh * B.ny, B.nxh * B.ny * B.nz};
    const bool masked = (MU < 3) && (tau > 1);
    const int slice = g.st;
    const int item = B.blk * (int)blockDim.x + (int)threadIdx.x;
    const bool active = item < B.n_items;
    if (!kQueue && !active) return;
    real* lb = links + B.link_off;
    const unsigned vh = (unsigned)B.vh;
    bool pending = false;
    RetryQ<real> mine{};
    if (active) {
        const int j = fdiv(item, slice, B.inv_slice);
        const int rem = item - (int)__umul24(j, slice);
        int t = j;
        if (masked) {
            if (tau == 2) {  // uniform: the thinnest slabs skip the division
                t = 2 * j + 1;
            } else {
                const int jt = fdiv(j, tau - 1, inv_tm1);
                t = jt * tau + 1 + (j - jt * (tau - 1));
            }
        }
        const int yz = fdiv(rem, g.sy, B.inv_nxh);
        const int xh = rem - (int)__umul24(yz, g.sy);
        const int z = fdiv(yz, g.ny, B.inv_ny);
        const int y = yz - (int)__umul24(z, g.ny);
        const int x = 2 * xh + ((y + z + t + parity) & 1);
        const Site c{x, y, z, t, (int)(__umul24(g.sy, yz) + __umul24(g.st, t))};

        // every load of the update is issued before any arithmetic
        const Site cpm = mv<MU, +1>(c, g);
        real v[3][6];
        gather_plane<real, MU, Nu<MU, 0>::v>(lb, vh, g, c, cpm, parity, v[0]);
        gather_plane<real, MU, Nu<MU, 1>::v>(lb, vh, g, c, cpm, parity, v[1]);
        gather_plane<real, MU, Nu<MU, 2>::v>(lb, vh, g, c, cpm, parity, v[2]);
        const unsigned self = ((MU * 2 + parity) * vh + (unsigned)(xh + c.hrow)) * (unsigned)sizeof(real);
        real old = real(0);
        if (KIND != 0) old = ldo(lb, self);
        real* dst = reinterpret_cast<real*>(reinterpret_cast<char*>(lb) + self);

        // the first Philox block depends only on the link's id and the counter:
        // formed here, it runs while the link angles are still in flight
        // canonical site x + Nx (y + Ny (z + Nz t)) = x + 2 hrow, so no multiplication
        const uint32_t lid = (uint32_t)MU + 4u * (uint32_t)x + 8u * (uint32_t)c.hrow;
        const uint32_t ctr = upd[B.res_index] + (uint32_t)pass_offset;
        Block4 b0;
        if (kQueue || KIND == 2)
            b0 = philox4x32_10(lid, ctr, 0u, KIND == 2 ? DOM_METRO : DOM_HB, E.seed, E.key_id);

        real ar, ai;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            real s, co;
            M<real>::sincos_(v[k][0] - v[k][1] - v[k][2], &s, &co);
            if (k == 0) {
                ar = co;
                ai = s;
            } else {
                ar += co;
                ai += s;
            }
            M<real>::sincos_(v[k][3] - v[k][4] - v[k][5], &s, &co);
            ar += co;
            ai += s;
        }
        if constexpr (KIND == 0) {
            const real R = M<real>::sqrt_(ar * ar + ai * ai);
            const real kappa = (real)E.beta * R;
            RetryQ<real> q;
            real th;
            bool done = true;
            if constexpr (sizeof(real) == 4) {
                // theta = psi - arg A as one angle: exp(i theta) is proportional to
                // exp(i psi) conj(A), so a single atan2 replaces arccos, atan2 and wrap
                q = RetryQ<float>{kappa, ar, ai, lid, self};
                if (kappa == 0.0f) {
                    // psi uniform from attempt 0: pi (2 U1 - 1), in revolutions U1 - 1/2
                    // (with A = 0 as well, theta = psi)
                    const float rev = M<float>::u1(b0.w[0]) - 0.5f;
                    if (R == 0.0f) q.ar = 1.0f;
                    th = hb_angle(q, __builtin_amdgcn_cosf(rev), __builtin_amdgcn_sinf(rev));
                } else {
                    done = hb_block(q, bf_env_f32(kappa), b0, &th);
                }
            } else {
                q = RetryQ<double>{kappa, ar, ai, lid, self};
                if (kappa == 0.0) {
                    // psi uniform from attempt 0: pi (2 U1 - 1) (with A = 0 as well, theta = psi)
                    double sp, cp;
                    sincos_bounded(M<double>::pi * (2.0 * M<double>::u1(b0.w[0]) - 1.0), &sp, &cp);
                    if (R == 0.0) q.ar = 1.0;
                    th = hb_angle(q, cp, sp);
                } else {
                    done = hb_block(q, bf_r_f64(kappa), b0, &th);
                }
            }
            if (done) {
                *dst = th;
            } else {
                pending = true;
                mine = q;
            }
        } else if (KIND == 2) {
            // Metropolis: theta' = theta + delta (2 U1 - 1), accepted when
            // U2 < exp(beta (Re(e^{i theta'} A) - Re(e^{i theta} A)))
            const Block4& b = b0;
            using m = M<real>;
            const real thn = wrap_angle<real>(old + (real)E.metro_delta * (real(2) * m::u1(b.w[0]) - real(1)));
            real sn, cn, so, co;
            m::sincos_(thn, &sn, &cn);
            m::sincos_(old, &so, &co);
            const real dl = (real)E.beta * ((ar * cn - ai * sn) - (ar * co - ai * so));
            if (dl >= real(0) || m::u2(b.w[1]) < m::exp_(dl)) *dst = thn;
        } else {
            // stored unconditionally (A = 0 writes the old angle back), so the
            // load of the old angle is issued with the staple loads
            const real phiA = M<real>::atan2_(ai, ar);
            const real th = wrap_angle<real>(-old - real(2) * phiA);
            *dst = (ar == real(0) && ai == real(0)) ? old : th;
        }
    }
    if constexpr (kQueue) {
        extern __shared__ __align__(16) unsigned char queue_bytes[];
        RetryQ<real>* queue = reinterpret_cast<RetryQ<real>*>(queue_bytes);
        __shared__ int wave_count[16];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const unsigned long long m = __ballot(pending);
        if (lane == 0) wave_count[wave] = __popcll(m);
        __syncthreads();
        int base = 0, total = 0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) {
            base += w < wave ? wave_count[w] : 0;
            total += wave_count[w];
        }
        if (pending) {
            const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
            queue[pos] = mine;
        }
        __syncthreads();
        const uint32_t ctr = upd[B.res_index] + (uint32_t)pass_offset;
        for (int i = threadIdx.x; i < total; i += blockDim.x) {
            const RetryQ<real> r = queue[i];
            const auto env = hb_env(r);
            real th = real(0);
            bool done = false;
            // attempts 2 .. 65535 (blocks 1 .. 32767); past the cap the link keeps its angle
            for (uint32_t jp = 1; jp < 32768u && !done; ++jp)
                done = hb_block(r, env, philox4x32_10(r.lid, ctr, jp, DOM_HB, E.seed, E.key_id), &th);
            if (done) *reinterpret_cast<real*>(reinterpret_cast<char*>(lb) + r.off) = th;
        }
    }
}

// With a start/stop event pair the launch goes through hipExtLaunchKernelGGL,
// whose events take the dispatch's own begin and end timestamps.
template <typename real, int KIND, int MU>
static void launch_update_mu(dim3 g, dim3 b, size_t lds, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                             const EnsDesc* d_ens, const UpdBlock* d_bmap, real* links, const uint32_t* d_upd,
                             int pass_offset, int parity, int tau, float inv_tm1)
{
    if (ev0)
        hipExtLaunchKernelGGL((k_update<real, KIND, MU>), g, b, lds, st, ev0, ev1, 0, d_ens, d_bmap, links, d_upd,
                              pass_offset, parity, tau, inv_tm1);
    else
        hipLaunchKernelGGL((k_update<real, KIND, MU>), g, b, lds, st, d_ens, d_bmap, links, d_upd, pass_offset,
                           parity, tau, inv_tm1);
}

template <typename real, int KIND>
static void launch_update_t(dim3 g, dim3 b, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, const EnsDesc* d_ens,
                            const UpdBlock* d_bmap, real* links, const uint32_t* d_upd, int pass_offset, int mu,
                            int parity, int tau, float inv_tm1)
{
    const size_t lds = KIND == 0 ? sizeof(RetryQ<real>) * b.x : 0;
    switch (mu) {
    case 0: launch_update_mu<real, KIND, 0>(g, b, lds, st, ev0, ev1, d_ens, d_bmap, links, d_upd, pass_offset, parity, tau, inv_tm1); break;
    case 1: launch_update_mu<real, KIND, 1>(g, b, lds, st, ev0, ev1, d_ens, d_bmap, links, d_upd, pass_offset, parity, tau, inv_tm1); break;
    case 2: launch_update_mu<real, KIND, 2>(g, b, lds, st, ev0, ev1, d_ens, d_bmap, links, d_upd, pass_offset, parity, tau, inv_tm1); break;
    default: launch_update_mu<real, KIND, 3>(g, b, lds, st, ev0, ev1, d_ens, d_bmap, links, d_upd, pass_offset, parity, tau, inv_tm1); break;
    }
}

hipError_t launch_update(const EnsDesc* d_ens, const UpdBlock* d_bmap, int total_blocks, int block, int precision,
                         void* links, const uint32_t* d_upd, int pass_offset, int kind, int mu, int parity, int tau,
                         hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop)
{
    if (total_blocks <= 0) return hipSuccess;
    if ((ev_start == nullptr) != (ev_stop == nullptr)) return hipErrorInvalidValue;
    const dim3 g(total_blocks), b(block);
    const float inv_tm1 = tau > 1 ? 1.0f / (float)(tau - 1) : 1.0f;
    if (kind < 0 || kind > 2) return hipErrorInvalidValue;
    if (precision == 0) {
        double* lk = (double*)links;
        if (kind == 0)
            launch_update_t<double, 0>(g, b, st, ev_start, ev_stop, d_ens, d_bmap, lk, d_upd, pass_offset, mu, parity, tau, inv_tm1);
        else if (kind == 1)
            launch_update_t<double, 1>(g, b, st, ev_start, ev_stop, d_ens, d_bmap, lk, d_upd, pass_offset, mu, parity, tau, inv_tm1);
        else
            launch_update_t<double, 2>(g, b, st, ev_start, ev_stop, d_ens, d_bmap, lk, d_upd, pass_offset, mu, parity, tau, inv_tm1);
    } else {
        float* lk = (float*)links;
        if (kind == 0)
            launch_update_t<float, 0>(g, b, st, ev_start, ev_stop, d_ens, d_bmap, lk, d_upd, pass_offset, mu, parity, tau, inv_tm1);
        else if (kind == 1)
            launch_update_t<float, 1>(g, b, st, ev_start, ev_stop, d_ens, d_bmap, lk, d_upd, pass_offset, mu, parity, tau, inv_tm1);
        else
            launch_update_t<float, 2>(g, b, st, ev_start, ev_stop, d_ens, d_bmap, lk, d_upd, pass_offset, mu, parity, tau, inv_tm1);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// All-link kernels: one work-item per (direction, parity, half site).
// ---------------------------------------------------------------------------
struct LinkItem {
    int dir, par, h, x, y, z, t;
};

__device__ inline bool decode_link(const EnsDesc& E, int item, LinkItem* o)
{
    if (item >= 8 * E.vh) return false;
    const int dp = item / E.vh;
    o->h = item - dp * E.vh;
    o->dir = dp >> 1;
    o->par = dp & 1;
    const int row = o->h / E.nxh;
    const int xh = o->h - row * E.nxh;
    const int yz = row;
    o->t = yz / (E.ny * E.nz);
    const int r2 = yz - o->t * E.ny * E.nz;
    o->z = r2 / E.ny;
    o->y = r2 - o->z * E.ny;
    o->x = 2 * xh + ((o->y + o->z + o->t + o->par) & 1);
    return true;
}

// Cold: theta = 0.  Hot: theta = pi (2u - 1), u = (w0 + 1/2) 2^-32 with w0 the
// first word of the Philox block (link id, 0, 0, INIT); formed in FP64 and
// rounded to the storage precision.
template <typename real>
__global__ void k_init(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart, int n_ens,
                       real* __restrict__ links, int start)
{
    const int bid = blockIdx.x;
    const int e = find_ens(bstart, n_ens, bid);
    const EnsDesc& E = ens[e];
    LinkItem it;
    if (!decode_link(E, (bid - bstart[e]) * (int)blockDim.x + (int)threadIdx.x, &it)) return;
    double th = 0.0;
    if (start) {
        const uint32_t lid = (uint32_t)(it.dir + 4 * (it.x + E.nx * (it.y + E.ny * (it.z + E.nz * it.t))));
        const Block4 b = philox4x32_10(lid, 0u, 0u, DOM_INIT, E.seed, E.key_id);
        const double u = ((double)b.w[0] + 0.5) * (1.0 / 4294967296.0);
        th = M<double>::pi * (2.0 * u - 1.0);
    }
    links[E.link_off + (size_t)(it.dir * 2 + it.par) * E.vh + it.h] = (real)th;
}

hipError_t launch_init_links(const EnsDesc* d_ens, const int* d_bstart_all, int n_ens, int total_blocks, int precision,
                             void* links, int start, hipStream_t st)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_init<double>, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart_all, n_ens,
                           (double*)links, start);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart_all, n_ens,
                           (float*)links, start);
    return hipGetLastError();
}

template <typename real>
__global__ void k_health(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart, int n_ens,
                         const real* __restrict__ links, unsigned long long* __restrict__ count)
{
    const int bid = blockIdx.x;
    const int e = find_ens(bstart, n_ens, bid);
    const EnsDesc& E = ens[e];
    LinkItem it;
    if (!decode_link(E, (bid - bstart[e]) * (int)blockDim.x + (int)threadIdx.x, &it)) return;
    const double th = (double)links[E.link_off + (size_t)(it.dir * 2 + it.par) * E.vh + it.h];
    const double lim = M<double>::pi * (1.0 + 1.0 / 1048576.0);
    if (!(th >= -lim && th <= lim)) atomicAdd(count, 1ull);
}

hipError_t launch_health(const EnsDesc* d_ens, const int* d_bstart_all, int n_ens, int total_blocks, int precision,
                         const void* links, unsigned long long* d_count, hipStream_t st)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_health<double>, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart_all, n_ens,
                           (const double*)links, d_count);
    else
        hipLaunchKernelGGL(k_health<float>, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart_all, n_ens,
                           (const float*)links, d_count);
    return hipGetLastError();
}

// Canonical FP64 view <-> even/odd storage, one ensemble at a time.
template <typename real>
__global__ void k_gather(const EnsDesc* __restrict__ ens, int e, const real* __restrict__ links,
                         double* __restrict__ canon, long long n_sites)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sites) return;
    const EnsDesc& E = ens[e];
    const int x = (int)(s % E.nx);
    long long r = s / E.nx;
    const int y = (int)(r % E.ny);
    r /= E.ny;
    const int z = (int)(r % E.nz);
    const int t = (int)(r / E.nz);
    const int par = (x + y + z + t) & 1;
    const int h = (x >> 1) + E.nxh * (y + E.ny * (z + E.nz * t));
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) canon[4 * s + mu] = (double)links[E.link_off + (size_t)(mu * 2 + par) * E.vh + h];
}

template <typename real>
__global__ void k_scatter(const EnsDesc* __restrict__ ens, int e, real* __restrict__ links,
                          const double* __restrict__ canon, long long n_sites)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sites) return;
    const EnsDesc& E = ens[e];
    const int x = (int)(s % E.nx);
    long long r = s / E.nx;
    const int y = (int)(r % E.ny);
    r /= E.ny;
    const int z = (int)(r % E.nz);
    const int t = (int)(r / E.nz);
    const int par = (x + y + z + t) & 1;
    const int h = (x >> 1) + E.nxh * (y + E.ny * (z + E.nz * t));
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) links[E.link_off + (size_t)(mu * 2 + par) * E.vh + h] = (real)canon[4 * s + mu];
}

hipError_t launch_gather_links(const EnsDesc* d_ens, int ens, int precision, const void* links, double* d_canon,
                               long long n_sites, hipStream_t st)
{
    const int g = (int)((n_sites + 255) / 256);
    if (precision == 0)
        hipLaunchKernelGGL(k_gather<double>, dim3(g), dim3(256), 0, st, d_ens, ens, (const double*)links, d_canon,
                           n_sites);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(g), dim3(256), 0, st, d_ens, ens, (const float*)links, d_canon,
                           n_sites);
    return hipGetLastError();
}

hipError_t launch_scatter_links(const EnsDesc* d_ens, int ens, int precision, void* links, const double* d_canon,
                                long long n_sites, hipStream_t st)
{
    const int g = (int)((n_sites + 255) / 256);
    if (precision == 0)
        hipLaunchKernelGGL(k_scatter<double>, dim3(g), dim3(256), 0, st, d_ens, ens, (double*)links, d_canon,
                           n_sites);
    else
        hipLaunchKernelGGL(k_scatter<float>, dim3(g), dim3(256), 0, st, d_ens, ens, (float*)links, d_canon, n_sites);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plaquette means per orientation (E_x, E_y, E_z, B_x, B_y, B_z), FP64 sums.
// Work-group (e, b), one of kPlaqBlocks per ensemble, walks the ensemble's
// sites in a fixed stride (V < 2^28 sites, so 32-bit indices) and reduces its
// sums through LDS; k_plaq_final adds an ensemble's partials in a fixed-order
// tree.
// ---------------------------------------------------------------------------
template <typename real>
__global__ void __launch_bounds__(256) k_plaq_partial(const EnsDesc* __restrict__ ens, const real* __restrict__ links,
                                                      double* __restrict__ partials)
{
    const int e = blockIdx.x / kPlaqBlocks;
    const int b = blockIdx.x % kPlaqBlocks;
    const EnsDesc& E = ens[e];
    LinkView<real> L{links + E.link_off, E.vh, E.nxh, E.ny, E.nz};
    const int V = 2 * E.vh;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    static const int pa[6] = {0, 1, 2, 1, 2, 0};
    static const int pb[6] = {3, 3, 3, 2, 0, 1};
    for (int s = b * 256 + (int)threadIdx.x; s < V; s += 256 * kPlaqBlocks) {
        const int x = s % E.nx;
        int r = s / E.nx;
        const int y = r % E.ny;
        r /= E.ny;
        const int z = r % E.nz;
        const int t = r / E.nz;
        const Coord c = {x, y, z, t};
        const int p = (x + y + z + t) & 1;
#pragma unroll
        for (int o = 0; o < 6; ++o) {
            const int a = pa[o], bb = pb[o];
            const Coord ca = step(c, a, +1, E.nx, E.ny, E.nz, E.nt);
            const Coord cb = step(c, bb, +1, E.nx, E.ny, E.nz, E.nt);
            const double th = (double)L.ld(a, p, c) + (double)L.ld(bb, p ^ 1, ca) - (double)L.ld(a, p ^ 1, cb) -
                              (double)L.ld(bb, p, c);
            acc[o] += cos(th);
        }
    }
    __shared__ double sh[6][256];
    for (int o = 0; o < 6; ++o) sh[o][threadIdx.x] = acc[o];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int o = 0; o < 6; ++o) sh[o][threadIdx.x] += sh[o][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) partials[(size_t)blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// one 256-thread work-group per ensemble: thread i adds partials i, i + 256,
// ... in order, then an LDS tree
__global__ void __launch_bounds__(256) k_plaq_final(const EnsDesc* __restrict__ ens,
                                                    const double* __restrict__ partials, double* __restrict__ out)
{
    const int e = blockIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < kPlaqBlocks; b += blockDim.x)
        for (int o = 0; o < 6; ++o) acc[o] += partials[((size_t)e * kPlaqBlocks + b) * 6 + o];
    __shared__ double sh[6][256];
    for (int o = 0; o < 6; ++o) sh[o][threadIdx.x] = acc[o];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int o = 0; o < 6; ++o) sh[o][threadIdx.x] += sh[o][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[e * 6 + threadIdx.x] = sh[threadIdx.x][0] / (2.0 * (double)ens[e].vh);
}

hipError_t launch_plaquette(const EnsDesc* d_ens, int n_ens, int, int precision, const void* links,
                            double* d_partials, double* d_out, hipStream_t st)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_plaq_partial<double>, dim3(n_ens * kPlaqBlocks), dim3(256), 0, st, d_ens,
                           (const double*)links, d_partials);
    else
        hipLaunchKernelGGL(k_plaq_partial<float>, dim3(n_ens * kPlaqBlocks), dim3(256), 0, st, d_ens,
                           (const float*)links, d_partials);
    hipLaunchKernelGGL(k_plaq_final, dim3(n_ens), dim3(256), 0, st, d_ens, d_partials, d_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free plaquette call: the per-work-group
// partial sums of up to kStaticPlaqEns ensembles (1.5 MiB), one copy per
// device for the life of the process.  Host code must not pass the array's
// name to a kernel: it reaches the array only through the address that
// hipGetSymbolAddress returns with the device current, kept per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[(size_t)kStaticPlaqEns * kPlaqBlocks * 6];

hipError_t static_scratch(double** ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double*>(p);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// RNG and sampler fills (bit-exact and statistical checks of the stream).
// ---------------------------------------------------------------------------
__global__ void k_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, size_t n,
                              uint32_t* __restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Block4 b = philox4x32_10(c0 + (uint32_t)i, c1, c2, c3, k0, k1);
    uint4 v;
    v.x = b.w[0];
    v.y = b.w[1];
    v.z = b.w[2];
    v.w = b.w[3];
    reinterpret_cast<uint4*>(out)[i] = v;
}

hipError_t launch_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, size_t n,
                              uint32_t* d_out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k0, k1, c0, c1, c2, c3, n,
                       d_out);
    return hipGetLastError();
}

template <typename real>
__global__ void k_vonmises_fill(real kappa, uint32_t seed, uint32_t key_id, uint32_t c0, uint32_t c1, size_t n,
                                double* __restrict__ out, int* __restrict__ att)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int na;
    const real psi = vonmises_psi<real>(kappa, seed, key_id, c0 + (uint32_t)i, c1, DOM_TEST, &na);
    out[i] = (double)psi;
    if (att) att[i] = na;
}

hipError_t launch_vonmises_fill(double kappa, int precision, uint32_t seed, uint32_t key_id, uint32_t c0, uint32_t c1,
                                size_t n, double* d_out, int* d_att, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 g((unsigned)((n + 255) / 256));
    if (precision == 0)
        hipLaunchKernelGGL(k_vonmises_fill<double>, g, dim3(256), 0, st, kappa, seed, key_id, c0, c1, n, d_out, d_att);
    else
        hipLaunchKernelGGL(k_vonmises_fill<float>, g, dim3(256), 0, st, (float)kappa, seed, key_id, c0, c1, n, d_out,
                           d_att);
    return hipGetLastError();
}

// the library's FP64 sine and cosine on given arguments
__global__ void k_sincos_fill(const double* __restrict__ x, size_t n, double* __restrict__ s, double* __restrict__ c)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sv, cv;
    sincos_bounded(x[i], &sv, &cv);
    s[i] = sv;
    c[i] = cv;
}

hipError_t launch_sincos_fill(const double* d_x, size_t n, double* d_s, double* d_c, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sincos_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d_x, n, d_s, d_c);
    return hipGetLastError();
}

// advances the counters of the n_ens ensembles described by ens[]
__global__ void k_advance(const EnsDesc* __restrict__ ens, uint32_t* __restrict__ upd, int n_ens, int delta)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n_ens) upd[ens[e].res_index] += (uint32_t)delta;
}

hipError_t launch_advance_counters(const EnsDesc* d_ens, uint32_t* d_upd, int n_ens, int delta, hipStream_t st)
{
    hipLaunchKernelGGL(k_advance, dim3((n_ens + 63) / 64), dim3(64), 0, st, d_ens, d_upd, n_ens, delta);
    return hipGetLastError();
}

}  // namespace u1ml
