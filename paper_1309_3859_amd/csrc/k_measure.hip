// k_measure.hip -- multilevel measurements, slab averages and slab products.
//
// Paper: Amado, Cardoso, Bicudo, arXiv 1309.3859.
//  - Sec. II.C.1: two-link operator T(x,t,r) = U_0^dagger(x,t) U_0(x+r mu,t); in
//    U(1) a product of two phases, so over a slab s of thickness tau
//    T^(tau)(x,s,r) = exp(-i Theta_s(x)) exp(i Theta_s(x + r mu)) with
//    Theta_s(x) = sum_{t in s} theta_t(x,t).
//  - Sec. II.C.2: slab averages [T^(2)] and their products; two levels
//    T^(4) = [T^(2)(t)] [T^(2)(t+2)].
//  - Sec. II.C.3: a^4 F^2 = 2 beta (1 - Re P), a^2 F = sqrt(beta) Im P,
//    TO^(2) = [T^(2) (O(t) + O(t+1))],
//    TO^(4) = [T^(2)(t)][TO^(2)(t+2)] + [TO^(2)(t)][T^(2)(t+2)],
//    <P^dagger P O> = 1/(N_sigma N_t |M|) sum_x sum_mu sum_S [TO](S)
//                      prod_{S' != S} [T](S').
//
// Design (instead of the paper's per-site running sums of every insertion,
// Sec. II.D): each inner measurement stores the slab phases exp(i Theta_s(x))
// and the slab sums of O for every plaquette orientation (the "history");
// at the end of the inner level one contraction pass forms every slab
// average in registers and writes it once.  Products over slabs are carried
// as (mantissa, binary exponent) pairs so they cannot underflow, and all sums
// over sites are double-double in a fixed order, so results are reproducible.
#include <type_traits>

#include "device_common.hpp"
#include "scaled.hpp"
#include "u1ml_internal.hpp"

namespace u1ml {

__device__ inline int find_ens_m(const int* __restrict__ bstart, int n_ens, int bid)
{
    int e = 0;
    while (e + 1 < n_ens && bid >= bstart[e + 1]) ++e;
    return e;
}

// ---------------------------------------------------------------------------
// double-double helpers (Knuth two-sum: additions only, immune to contraction)
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};

__device__ inline dd dd_add(dd a, double b)
{
    const double s = a.hi + b;
    const double bb = s - a.hi;
    const double err = (a.hi - (s - bb)) + (b - bb) + a.lo;
    const double hi = s + err;
    return dd{hi, err - (hi - s)};
}

__device__ inline dd dd_add(dd a, dd b)
{
    const double s = a.hi + b.hi;
    const double bb = s - a.hi;
    const double err = (a.hi - (s - bb)) + (b.hi - bb) + a.lo + b.lo;
    const double hi = s + err;
    return dd{hi, err - (hi - s)};
}

// absolute orientation of frame component c for charge axis dir:
// E_i -> i (plaquette P_{i t}); B_x, B_y, B_z -> 3, 4, 5 (P_yz, P_zx, P_xy)
__device__ inline int comp_orient(int c, int dir) { return c < 3 ? (dir + c) % 3 : 3 + (dir + c - 3) % 3; }
__device__ inline bool comp_spans_axis(int c) { return c == 0 || c == 4 || c == 5; }

// ---------------------------------------------------------------------------
// Fill kernel (used instead of memset so that captured graphs replay cleanly)
// ---------------------------------------------------------------------------
__global__ void k_zero(uint4* __restrict__ p, size_t n16)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    size_t g = (n16 + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(256), 0, st, (uint4*)p, n16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Measurement m of a configuration (one work-item per spatial site x and slab s
// of the innermost level):
//   hist_c[m_in][s][x]       = exp(i Theta_s(x)), Theta_s(x) = sum_{t in s} theta_t(x, t)
//   (multihit) at hcm_off: prod_{t in s} of the temporal links' conditional means
//   hist_o[m_in][s][2o+k][x] = sum_{t in s} O_k(P_o(x, t)); k = 0: 2 beta (1 - cos),
//                              k = 1: sqrt(beta) sin, orientations o = P_xt, P_yt,
//                              P_zt, P_yz, P_zx, P_xy
//   vac_part[block][2o+k]    += block sum of O_k over every plaquette (vacuum <O>),
//                              double-double, measurements in order
// m_in indexes the measurement inside the innermost level, m the measurement
// inside the configuration.
// ---------------------------------------------------------------------------
// Slab sums of the two insertion kinds of one plaquette orientation,
// accumulated over the slab's time slices and read out once.
template <typename real>
struct SlabO;

template <>
struct SlabO<double> {
    double sq = 0.0, lin = 0.0;
    __device__ inline void add(double th, double beta, double sqrt_beta)
    {
        double s, c;
        sincos_bounded(th, &s, &c);
        sq += 2.0 * beta * (1.0 - c);
        lin += sqrt_beta * s;
    }
    __device__ inline double osq(double) const { return sq; }
    __device__ inline double olin(double) const { return lin; }
};

template <>
struct SlabO<float> {
    // 1 - cos(th) = 2 sin^2(th / 2), free of cancellation in FP32; the FP32
    // sums of sin^2(th / 2) and sin(th) over the slab's few slices are scaled
    // by 4 beta and sqrt(beta) in FP64
    float sh2 = 0.0f, s = 0.0f;
    __device__ inline void add(float th, double, double)
    {
        const float rev = th * 0.159154943f;
        const float sh = __builtin_amdgcn_sinf(0.5f * rev);
        sh2 += sh * sh;
        s += __builtin_amdgcn_sinf(rev);
    }
    __device__ inline double osq(double beta) const { return 4.0 * beta * (double)sh2; }
    __device__ inline double olin(double sqrt_beta) const { return sqrt_beta * (double)s; }
};

// Sum of 12 per-thread doubles over a 256-thread block in a fixed order (lanes
// l and l + 32 of a wave added by one exchange, the 128 pair sums staged in
// LDS, then each wave reduces three of the quantities), added to the block's
// running double-double partials acc[12][2] of the configuration; the first
// measurement (first != 0) overwrites them instead, so they need no clearing
// between configurations.  12 KB of LDS, so that LDS does not limit a CU to
// fewer work-groups than its wave slots hold.
__device__ inline void block_sum12(const double* v, double* acc, int first)
{
    __shared__ double red[12][128];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double a = v[k] + __shfl_xor(v[k], 32);
        if (lane < 32) red[k][wave * 32 + lane] = a;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        const int k = 3 * wave + kk;
        double a = red[k][lane] + red[k][lane + 64];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        if (lane == 0) {
            const dd r = first ? dd{a, 0.0} : dd_add(dd{acc[2 * k], acc[2 * k + 1]}, a);
            acc[2 * k] = r.hi;
            acc[2 * k + 1] = r.lo;
        }
    }
}

template <typename real, bool MULTIHIT>
__global__ void __launch_bounds__(256) k_measure(const EnsDesc* __restrict__ ens, const int2* __restrict__ bmap,
                                                 const real* __restrict__ links, double2* __restrict__ hist_c,
                                                 real* __restrict__ hist_o, double* __restrict__ vac_part, int m_in,
                                                 int m, int tau, int store_o, int n_blocks)
{
    // XCD-aware order: the hardware deals consecutive work-groups to the eight
    // XCDs in turn, so work-group b takes block (b mod 8) G/8 + b/8 of the map
    // (G, a multiple of 8, launched): each XCD measures a contiguous run of
    // sites and finds the neighbours' links in its own L2
    const int bid = (int)(blockIdx.x & 7u) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
    if (bid >= n_blocks) return;  // uniform: padding of the launch to a multiple of 8
    const int2 be = bmap[bid];
    const EnsDesc& E = ens[be.x];
    const int nsig = E.nsig, S = E.s_in;
    const int item = be.y * 256 + (int)threadIdx.x;
    const real* lb = links + E.link_off;
    const unsigned vh = (unsigned)E.vh;
    constexpr unsigned w = sizeof(real);
    double vac[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) vac[k] = 0.0;
    if (item < nsig * S) {
        const Geo g{E.nx, E.ny, E.nz, E.nt, E.nxh, E.nxh * E.ny, E.nxh * E.ny * E.nz};
        // division-free decode; N_sigma is even, so item / N_sigma = (item / 2) / (N_sigma / 2)
        // with the divisor N_sigma / 2 (the slice) inside fdiv's 24-bit range, and
        // 1/Nx = (1/(Nx/2)) / 2 exactly
        const int s = fdiv(item >> 1, nsig >> 1, E.inv_slice);
        const int xs = item - s * nsig;
        const int yz = fdiv(xs, E.nx, 0.5f * E.inv_nxh);
        const int x = xs - yz * E.nx;
        const int z = fdiv(yz, E.ny, E.inv_ny);
        const int y = yz - z * E.ny;
        double Th = 0.0;
        double2 cm = make_double2(1.0, 0.0);  // multihit slab phase
        SlabO<real> so[6];
        Site c{x, y, z, s * tau, g.sy * yz + g.st * (s * tau)};
        // the 16 link angles of the six plaquettes at (x, t): u[0..3] the four
        // links at the site, then the ones at x + x, x + y, x + z, x + t
        auto load_slice = [&](const Site& c, real* u) {
            // element offsets of the site's parity and the other one (a select,
            // not a multiplication by the per-thread parity)
            const bool odd = ((x + y + z + c.t) & 1) != 0;
            const unsigned po = odd ? vh : 0u, qo = odd ? 0u : vh;
            const Site cx = mv<0, +1>(c, g), cy = mv<1, +1>(c, g), cz = mv<2, +1>(c, g), ct = mv<3, +1>(c, g);
            auto L = [&](unsigned dir, unsigned par_off, const Site& st) {
                return ldo(lb, (dir * 2u * vh + par_off + hidx(st)) * w);
            };
            u[0] = L(0, po, c), u[1] = L(1, po, c), u[2] = L(2, po, c), u[3] = L(3, po, c);
            u[4] = L(3, qo, cx), u[5] = L(3, qo, cy), u[6] = L(3, qo, cz);   // t-links at x + x, x + y, x + z
            u[7] = L(0, qo, ct), u[8] = L(1, qo, ct), u[9] = L(2, qo, ct);   // x, y, z-links at x + t
            u[10] = L(2, qo, cy), u[11] = L(1, qo, cz);                       // z at x + y, y at x + z
            u[12] = L(0, qo, cz), u[13] = L(2, qo, cx);                       // x at x + z, z at x + x
            u[14] = L(1, qo, cx), u[15] = L(0, qo, cy);                       // y at x + x, x at x + y
        };
        auto use_slice = [&](const Site& c, const real* u) {
            Th += (double)u[3];
            if (MULTIHIT) {
                // conditional mean of the temporal link: e^{-i arg A} I1/I0(beta |A|)
                real ar, ai;
                const int p = ((x + y + z + c.t) & 1);
                staple_sum<real, 3>(lb, vh, g, c, p, &ar, &ai);
                const double R = sqrt((double)ar * (double)ar + (double)ai * (double)ai);
                const double f = R > 0.0 ? bessel_ratio(E.beta * R) / R : 0.0;
                const double ur = (double)ar * f, ui = -(double)ai * f;
                cm = make_double2(cm.x * ur - cm.y * ui, cm.x * ui + cm.y * ur);
            }
            real th[6];
            th[0] = u[0] + u[4] - u[7] - u[3];   // P_xt
            th[1] = u[1] + u[5] - u[8] - u[3];   // P_yt
            th[2] = u[2] + u[6] - u[9] - u[3];   // P_zt
            th[3] = u[1] + u[10] - u[11] - u[2]; // P_yz
            th[4] = u[2] + u[12] - u[13] - u[0]; // P_zx
            th[5] = u[0] + u[14] - u[15] - u[1]; // P_xy
#pragma unroll
            for (int o = 0; o < 6; ++o) so[o].add(th[o], E.beta, E.sqrt_beta);
        };
        // slices two at a time, all 32 loads issued before either is used
        int k = 0;
        for (; k + 1 < tau; k += 2) {
            const Site c1 = mv<3, +1>(c, g);
            real a[16], b[16];
            load_slice(c, a);
            load_slice(c1, b);
            use_slice(c, a);
            use_slice(c1, b);
            c = mv<3, +1>(c1, g);
        }
        if (k < tau) {
            real a[16];
            load_slice(c, a);
            use_slice(c, a);
        }
        double os[12];
#pragma unroll
        for (int o = 0; o < 6; ++o) {
            os[2 * o] = so[o].osq(E.beta);
            os[2 * o + 1] = so[o].olin(E.sqrt_beta);
        }
        double sn, cs;
        sincos_bounded(Th, &sn, &cs);  // |Th| <= tau pi
        hist_c[E.hc_off + ((size_t)m_in * S + s) * nsig + xs] = make_double2(cs, sn);
        if (MULTIHIT) hist_c[E.hcm_off + ((size_t)m_in * S + s) * nsig + xs] = cm;
        if (store_o) {
            // per-measurement slab sums are stored in the link precision; the sums
            // over measurements are formed in FP64 by the contraction
            real* ho = hist_o + E.ho_off + ((size_t)m_in * S + s) * 12 * nsig + xs;
#pragma unroll
            for (int k = 0; k < 12; ++k) ho[(size_t)k * nsig] = (real)os[k];
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) vac[k] = os[k];
    }
    block_sum12(vac, vac_part + E.vac_part_off + (size_t)be.y * 24, m == 0);
}

hipError_t launch_measure(const EnsDesc* d_ens, const int2* d_bmap, int total_blocks, int precision, const void* links,
                          double2* hist_c, void* hist_o, double* vac_part, int m_in, int m, int tau, int store_o,
                          int multihit, hipStream_t st)
{
    if (total_blocks <= 0) return hipSuccess;
    const dim3 g((total_blocks + 7) / 8 * 8), b(256);
    if (precision == 0) {
        const double* l = (const double*)links;
        if (multihit)
            hipLaunchKernelGGL((k_measure<double, true>), g, b, 0, st, d_ens, d_bmap, l, hist_c, (double*)hist_o,
                               vac_part, m_in, m, tau, store_o, total_blocks);
        else
            hipLaunchKernelGGL((k_measure<double, false>), g, b, 0, st, d_ens, d_bmap, l, hist_c, (double*)hist_o,
                               vac_part, m_in, m, tau, store_o, total_blocks);
    } else {
        const float* l = (const float*)links;
        if (multihit)
            hipLaunchKernelGGL((k_measure<float, true>), g, b, 0, st, d_ens, d_bmap, l, hist_c, (float*)hist_o,
                               vac_part, m_in, m, tau, store_o, total_blocks);
        else
            hipLaunchKernelGGL((k_measure<float, false>), g, b, 0, st, d_ens, d_bmap, l, hist_c, (float*)hist_o,
                               vac_part, m_in, m, tau, store_o, total_blocks);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inner-level correlator averages, for charge axis mu and slab s (c_m: stored
// slab phases of measurement m):
//   [T](s,x,r) = 1/n sum_m conj(c_m(x)) c_m(x + r mu)
// Everything a pair (x, r) reads lies on its own line parallel to mu.  A group
// of threads owns one line, one thread per pair (x, r); the line's phases are
// staged through LDS in chunks of measurements, so memory delivers each
// history element once per line rather than once per separation.  The sums
// over measurements run in order m = 0, 1, ... in every thread.
// Launch: grid (work-groups of the ensembles' lines, slab, axis); a
// work-group holds E.con_lpb lines of blockDim / con_lpb threads each.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(512) k_contract(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                   int n_ens, const ObsDesc* __restrict__ obs,
                                                   const int* __restrict__ rlist, const double2* __restrict__ hist_c,
                                                   double2* __restrict__ avg_t, int n_meas)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int e = find_ens_m(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int S = E.s_in, s = blockIdx.y;
    if (s >= S) return;  // uniform for the block
    const int id = blockIdx.z, dir = O.dirs[id];
    const int n3[3] = {E.nx, E.ny, E.nz};
    const int N = n3[dir];
    const int d1 = dir == 2 ? 0 : dir + 1, d2 = dir == 0 ? 2 : dir - 1;  // (dir + 1) % 3, (dir + 2) % 3
    const int nsig = E.nsig;
    const int nlines = nsig / N;
    const int lpb = E.con_lpb, G = (int)blockDim.x / lpb;
    const int grp = (int)threadIdx.x / G, lane = (int)threadIdx.x - grp * G;
    const int line = (blockIdx.x - bstart[e]) * lpb + grp;
    if ((blockIdx.x - bstart[e]) * lpb >= nlines) return;  // whole block past this axis' lines (uniform)
    const bool line_ok = line < nlines;
    const int mc = E.con_mc;
    const int nmax = max(E.nx, max(E.ny, E.nz));
    const int row_len = mc * nmax;  // LDS elements of one staged row of one line
    const int nc_rows = O.multihit ? 2 : 1;  // plain phases, and multihit phases
    // LDS, site index k fastest, so that the consecutive pairs (x, r) of a
    // wave read consecutive 16-byte words (no bank conflicts):
    //   cl[q][k], clm[q][k]        phases of site k of the line (double2)
    double2* cl = reinterpret_cast<double2*>(lds_raw) + (size_t)grp * row_len;
    double2* clm = reinterpret_cast<double2*>(lds_raw) + (size_t)(nc_rows - 1) * lpb * row_len + (size_t)grp * row_len;

    // transverse coordinates of the line; sites along it are `stride` apart
    const int a1 = line_ok ? line % n3[d1] : 0, a2 = line_ok ? line / n3[d1] : 0;
    const int stride = dir == 0 ? 1 : (dir == 1 ? E.nx : E.nx * E.ny);
    auto site0 = [&](int o1, int o2) {  // line position 0, displaced by (o1, o2) across the axis
        int c[3];
        c[dir] = 0;
        c[d1] = ((a1 + o1) % n3[d1] + n3[d1]) % n3[d1];
        c[d2] = ((a2 + o2) % n3[d2] + n3[d2]) % n3[d2];
        return c[0] + E.nx * (c[1] + E.ny * c[2]);
    };
    const int base = site0(0, 0);
    const size_t mstride = (size_t)S * nsig;
    const double2* hc = hist_c + E.hc_off + (size_t)s * nsig + base;
    const double2* hcm = hist_c + E.hcm_off + (size_t)s * nsig + base;
    const double inv = 1.0 / (double)n_meas;
    const int nr = O.n_r, pairs = N * nr;
    const int npass = (pairs + G - 1) / G;

    // element j of a staged block (row, q, k), k fastest (contiguous in the
    // history for the x axis), carried from lane to lane + G without a
    // division per element
    const int g_q = G / N, g_k = G - (G / N) * N;
    const int l_q = lane / N, l_k = lane - (lane / N) * N;
    auto stage_rows = [&](const double2* src, double2* dst, int m0, int mm) {
        int q = l_q, k = l_k;
        for (int j = lane; j < mm * N; j += G) {
            dst[q * N + k] = src[(size_t)(m0 + q) * mstride + (size_t)k * stride];
            q += g_q;
            k += g_k;
            if (k >= N) {
                k -= N;
                ++q;
            }
        }
    };

    for (int pass = 0; pass < npass; ++pass) {
        const int pr = pass * G + lane;
        const bool act = line_ok && pr < pairs;
        const int ir = act ? pr / N : 0;
        const int x = act ? pr - ir * N : 0;
        const int r_ir = rlist[ir];  // 1 <= r < N
        int xr = x + r_ir;
        if (xr >= N) xr -= N;
        // multihit: both ends from the multihit phases, except neighbours on
        // the periodic axis (their temporal links share plaquettes): there
        // the far end keeps the plain phase
        const double2* pa = (O.multihit ? clm : cl) + x;
        const double2* pb = ((O.multihit && r_ir != 1 && r_ir != N - 1) ? clm : cl) + xr;
        double tre = 0.0, tim = 0.0;
        for (int m0 = 0; m0 < n_meas; m0 += mc) {
            const int mm = min(mc, n_meas - m0);
            __syncthreads();
            if (line_ok) {
                stage_rows(hc, cl, m0, mm);
                if (O.multihit) stage_rows(hcm, clm, m0, mm);
            }
            __syncthreads();
            if (act) {
#pragma unroll 4
                for (int q = 0; q < mm; ++q) {
                    const double2 a = pa[q * N], b = pb[q * N];
                    tre += a.x * b.x + a.y * b.y;
                    tim += a.x * b.y - a.y * b.x;
                }
            }
        }
        if (act)
            avg_t[E.at_off + (((size_t)id * nr + ir) * S + s) * nsig + base + (size_t)x * stride] =
                make_double2(tre * inv, tim * inv);
    }
}

// ---------------------------------------------------------------------------
// Insertion averages of the inner level (history form), for charge axis mu and
// slab s:
//   [TO](s, x, r, p, c, k) = 1/n sum_m T_m(s, x, r) O_m(x + sh(r, p, c) + p_perp, o(c), k),
//   T_m(x, r) = conj(c_m(x)) c_m(x + r mu),
// sh = l + (mode ? floor((r-1)/2) or floor(r/2) : 0) (the probe's offset along
// the axis, the mid-plane term depending on whether the component's plaquette
// spans mu).  The (probe, component) slots with the same (l, mode, spans) meet
// every T value at the same offset, so they are grouped in blocks of KS
// slots: the O pair at position y of a slot's displaced line pairs with
// T(y - sh(r), r) for every r, and work-item (y, r-block, slot block) keeps
// KR x KS x 4 accumulators.  Per measurement it forms its KR values of T from
// two staged phases each (no separate T pass) and reads one O pair per slot
// from LDS, converting it to FP64 there.  Work-group: one line of the axis,
// one slab, ins_pbw slot blocks; per chunk of ins_mc measurements it stages
// the line's phases and the O rows of its slots (16-byte loads where the line
// is contiguous in memory).  Sums over measurements run in order m = 0, 1, ...
// for every output.
// Launch: grid (work-groups of the ensembles' lines x slot-block chunks, slab,
// axis), up to kInsThreads work-items.
// ---------------------------------------------------------------------------
template <typename ot, int V>
__device__ inline void stage_o_rows(ot* __restrict__ ol, const ot* __restrict__ ho, const int* __restrict__ rowoff,
                                    int mm, int nrows, int N, int stride, size_t mstride_o, int m0)
{
    // vectors of V elements along y: ((q nrows + row) nv + v), walked with a carry
    const int nv = N / V, per_q = nrows * nv, total = mm * per_q;
    const int B = blockDim.x;
    const int dq = B / per_q, drem = B - dq * per_q;
    int f = threadIdx.x;
    int q = f / per_q, rem = f - q * per_q;
    constexpr int U = 4;  // vectors per work-item and round, all loads before any store
    using vec = typename std::conditional<V == 1, ot, typename std::conditional<sizeof(ot) == 4, float4, double2>::type>::type;
    while (f < total) {
        vec v[U];
        int dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dst[u] = -1;
            if (f < total) {
                const int row = rem / nv, iv = rem - row * nv;
                const int off = rowoff[row];
                const size_t ob = (size_t)(m0 + q) * mstride_o + (size_t)off;
                if constexpr (V == 1) {
                    v[u] = off >= 0 ? ho[ob + (size_t)iv * stride] : ot(0);
                } else {
                    v[u] = off >= 0 ? *reinterpret_cast<const vec*>(ho + ob + (size_t)iv * V) : vec{};
                }
                dst[u] = (q * nrows + row) * N + iv * V;
            }
            f += B;
            q += dq;
            rem += drem;
            if (rem >= per_q) {
                rem -= per_q;
                ++q;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (dst[u] >= 0) *reinterpret_cast<vec*>(ol + dst[u]) = v[u];
    }
}

template <typename ot, int KR, int KS, int NC>
__global__ void __launch_bounds__(kInsThreads, 2) k_contract_ins(
    const EnsDesc* __restrict__ ens, const int* __restrict__ bstart, int n_ens, const ObsDesc* __restrict__ obs,
    const int* __restrict__ rlist, const int* __restrict__ comps, const int* __restrict__ sblk,
    const double2* __restrict__ hist_c, const ot* __restrict__ hist_o, double2* __restrict__ avg_to, int n_meas,
    int n_blocks)
{
    // two chunk buffers as separate LDS objects, so that the compiler can tell
    // the copies into one from the reads of the other (no wait between them)
    __shared__ double2 lph0[kInsPh], lph1[kInsPh];                            // phases [q][x]
    __shared__ __align__(16) unsigned char lo0[kInsOb], lo1[kInsOb];          // O rows [q][row][y]
    __shared__ int rowoff[kInsRowsMax];  // each O row's element offset within one (measurement, slab) block, -1: empty slot
    // XCD-aware order: the hardware deals consecutive work-groups to the eight
    // XCDs in turn, so work-group b takes logical block (b mod 8) G/8 + b/8
    // (G, a multiple of 8, launched); each XCD then sums a contiguous run of
    // lines, whose displaced O lines overlap, from its own L2
    const int bid = (int)(blockIdx.x & 7u) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
    if (bid >= n_blocks) return;  // uniform: padding of the launch to a multiple of 8
    const int e = find_ens_m(bstart, n_ens, bid);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int S = E.s_in, s = blockIdx.y;
    if (s >= S) return;  // uniform for the block
    const int id = blockIdx.z;
    const int dir = O.dirs[id];
    const int n3[3] = {E.nx, E.ny, E.nz};
    const int N = NC ? NC : n3[dir];  // NC: every line of the launch has NC sites (constant LDS offsets)
    const int d1 = dir == 2 ? 0 : dir + 1, d2 = dir == 0 ? 2 : dir - 1;  // (dir + 1) % 3, (dir + 2) % 3
    const int nsig = E.nsig, nlines = nsig / N;
    const int nr = O.n_r, nrb = (nr + KR - 1) / KR;
    const int nsb = O.n_pblocks, bpw = E.ins_pbw, nchunk = (nsb + bpw - 1) / bpw;
    const int local = bid - bstart[e];
    const int line = local / nchunk, chunk = local - line * nchunk;
    if (line >= nlines) return;  // uniform: this axis has fewer lines than the ensemble's largest
    const int sb0 = chunk * bpw, nbw = min(bpw, nsb - sb0);
    const int nrows = nbw * KS * 2;  // O rows of one measurement: (slot block, slot, kind)
    const int mc = E.ins_mc;


    const int a1 = line % n3[d1], a2 = line / n3[d1];
    const int stride = dir == 0 ? 1 : (dir == 1 ? E.nx : E.nx * E.ny);
    auto site0 = [&](int o1, int o2) {  // line position 0, displaced by (o1, o2) across the axis
        int c[3];
        c[dir] = 0;
        c[d1] = ((a1 + o1) % n3[d1] + n3[d1]) % n3[d1];
        c[d2] = ((a2 + o2) % n3[d2] + n3[d2]) % n3[d2];
        return c[0] + E.nx * (c[1] + E.ny * c[2]);
    };
    const int base = site0(0, 0);
    const size_t mstride = (size_t)S * nsig;
    const size_t mstride_o = (size_t)S * 12 * nsig;
    const double2* hc = hist_c + E.hc_off + (size_t)s * nsig + base;
    const ot* ho = hist_o + E.ho_off + (size_t)s * 12 * nsig;
    const double inv = 1.0 / (double)n_meas;
    const int tid = threadIdx.x;
    for (int j = tid; j < nrows; j += blockDim.x) {
        const int bl = j / (2 * KS), rem = j - bl * 2 * KS, k = rem >> 1, kind = rem & 1;
        const int* B = sblk + kInsBlkInts * (sb0 + bl);
        int off = -1;
        if (k < B[3]) {
            const int* sl = B + 4 + 4 * k;  // probe, component index, p1, p2
            off = (2 * comp_orient(comps[sl[1]], dir) + kind) * nsig + site0(sl[2], sl[3]);
        }
        rowoff[j] = off;
    }
    // A line contiguous in memory (the x axis) with N a multiple of the
    // 16-byte vector: every row offset is then a multiple of the vector
    // (a line starts at a multiple of Nx, rows at multiples of nsig), and
    // each wave copies 64 vectors of a chunk straight from memory into LDS
    // (global_load_lds), so the next chunk streams in while this one is
    // summed.  Otherwise the chunk is staged through registers.
    constexpr int VW = 16 / (int)sizeof(ot);
    const bool dma = stride == 1 && N % VW == 0 && (reinterpret_cast<uintptr_t>(ho) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(hc) & 15) == 0;
    const int nv = N / VW, per_q = nrows * nv;
    const int lane = tid & 63, wv = tid >> 6, nw = ((int)blockDim.x + 63) >> 6;
    // this lane's first O vector of a chunk and the step between its spans, as (q, row, iv)
    const int ostep = nw * 64;
    const int odq = ostep / per_q, odrem = ostep - odq * per_q;
    const int odrow = odrem / nv, odiv = odrem - odrow * nv;
    const int ou0 = wv * 64 + lane, oq0 = ou0 / per_q, orem0 = ou0 - oq0 * per_q;
    const int orow0 = orem0 / nv, oiv0 = orem0 - orow0 * nv;
    auto issue = [&](int m0, int mm, double2* php, unsigned char* op) {
        // phases: vector v = q N + x
        for (int j = wv; j * 64 < mm * N; j += nw) {
            const int v = j * 64 + lane;
            if (v < mm * N) {
                const int q = v / N, x = v - q * N;
                __builtin_amdgcn_global_load_lds((const void*)(hc + (size_t)(m0 + q) * mstride + x),
                                                 (__attribute__((address_space(3))) void*)(php + j * 64), 16, 0, 0);
            }
        }
        // O rows: vector u = (q nrows + row) nv + iv
        int q = oq0, row = orow0, iv = oiv0;
        for (int j = wv; j * 64 < mm * per_q; j += nw) {
            if (q < mm) {
                const int off = rowoff[row];
                if (off >= 0)
                    __builtin_amdgcn_global_load_lds((const void*)(ho + (size_t)(m0 + q) * mstride_o + off + iv * VW),
                                                     (__attribute__((address_space(3))) void*)(op + (size_t)j * 1024),
                                                     16, 0, 0);
            }
            q += odq;
            iv += odiv;
            if (iv >= nv) {
                iv -= nv;
                ++row;
            }
            row += odrow;
            if (row >= nrows) {
                row -= nrows;
                ++q;
            }
        }
    };
    // phases of a chunk through registers, [q][x]: this work-item's first element and its step
    const int k0 = tid % N, q0 = tid / N, dqp = (int)blockDim.x / N, dkp = (int)blockDim.x - dqp * N;
    auto stage = [&](int m0, int mm, double2* ph, unsigned char* op) {
        int q = q0, k = k0;
        while (q < mm) {
            ph[q * N + k] = hc[(size_t)(m0 + q) * mstride + (size_t)k * stride];
            q += dqp;
            k += dkp;
            if (k >= N) {
                k -= N;
                ++q;
            }
        }
        stage_o_rows<ot, 1>(reinterpret_cast<ot*>(op), ho, rowoff, mm, nrows, N, stride, mstride_o, m0);
    };

    const int ntask = nbw * nrb * N;
    const int nch = (n_meas + mc - 1) / mc;
    for (int t0 = 0; t0 < ntask; t0 += blockDim.x) {
        const int task = t0 + tid;
        const bool act = task < ntask;
        const int y = act ? task % N : 0;
        const int rest = task / N;
        const int rb = act ? rest % nrb : 0, bl = act ? rest / nrb : 0;
        const int* B = sblk + kInsBlkInts * (sb0 + min(bl, nbw - 1));
        const int l = B[0], mode = B[1], spans = B[2], ns = B[3];
        // positions of T(y - sh(r), r): x and x + r of each of the work-item's separations
        int xa[KR], xb[KR];
#pragma unroll
        for (int j = 0; j < KR; ++j) {
            const int r = rlist[min(rb * KR + j, nr - 1)];
            const int sh = l + (mode ? (spans ? (r - 1) / 2 : r / 2) : 0);
            int x = (y - sh) % N;
            x += x < 0 ? N : 0;
            xa[j] = x;
            xb[j] = (x + r) % N;
        }
        double acc[KR][KS][4];
#pragma unroll
        for (int j = 0; j < KR; ++j)
#pragma unroll
            for (int k = 0; k < KS; ++k)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[j][k][q] = 0.0;

        // the sums over chunk ci (measurements ci mc, ...) from one buffer pair
        auto sum_chunk = [&](const double2* ph, const unsigned char* op, int ci) {
            if (!act) return;
            const int mm = min(mc, n_meas - ci * mc);
            const ot* ob = reinterpret_cast<const ot*>(op) + (size_t)bl * 2 * KS * N + y;
            for (int q = 0; q < mm; ++q) {
                const double2* pq = ph + q * N;
                double2 t[KR];
#pragma unroll
                for (int j = 0; j < KR; ++j) {
                    const double2 a = pq[xa[j]], b = pq[xb[j]];
                    t[j] = make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
                }
                const ot* oq = ob + (size_t)q * nrows * N;
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const double o0 = (double)oq[(2 * k) * N], o1 = (double)oq[(2 * k + 1) * N];
#pragma unroll
                    for (int j = 0; j < KR; ++j) {
                        acc[j][k][0] += t[j].x * o0;
                        acc[j][k][1] += t[j].y * o0;
                        acc[j][k][2] += t[j].x * o1;
                        acc[j][k][3] += t[j].y * o1;
                    }
                }
            }
        };
        __syncthreads();  // row offsets written; the previous pass done with both buffers
        if (dma) {
            // chunk ci streams into lph0/lo0 (even ci) or lph1/lo1 (odd ci) while the
            // previous one is summed; before a buffer is summed, this wave's
            // copies into it have landed (vmcnt 0) and the barrier makes every
            // wave's visible and ends the sums over the chunk before, whose
            // buffer the next copies overwrite
            issue(0, min(mc, n_meas), lph0, lo0);
            for (int ci = 0; ci < nch; ci += 2) {
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
                __syncthreads();
                if (ci + 1 < nch) issue((ci + 1) * mc, min(mc, n_meas - (ci + 1) * mc), lph1, lo1);
                sum_chunk(lph0, lo0, ci);
                if (ci + 1 >= nch) break;
                __builtin_amdgcn_s_waitcnt(0x0F70);
                __syncthreads();
                if (ci + 2 < nch) issue((ci + 2) * mc, min(mc, n_meas - (ci + 2) * mc), lph0, lo0);
                sum_chunk(lph1, lo1, ci + 1);
            }
        } else {
            for (int ci = 0; ci < nch; ++ci) {
                if (ci > 0) __syncthreads();
                stage(ci * mc, min(mc, n_meas - ci * mc), lph0, lo0);
                __syncthreads();
                sum_chunk(lph0, lo0, ci);
            }
        }
        if (act) {
#pragma unroll
            for (int j = 0; j < KR; ++j) {
                const int ir = rb * KR + j;
                if (ir >= nr) continue;
                const size_t xs = (size_t)base + (size_t)xa[j] * stride;
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    if (k >= ns) continue;
                    const int p = B[4 + 4 * k], ic = B[5 + 4 * k];
                    const size_t kq = ((((size_t)id * nr + ir) * O.n_probe + p) * O.n_comp + ic) * 2;
                    avg_to[E.ato_off + ((kq + 0) * S + s) * nsig + xs] =
                        make_double2(acc[j][k][0] * inv, acc[j][k][1] * inv);
                    avg_to[E.ato_off + ((kq + 1) * S + s) * nsig + xs] =
                        make_double2(acc[j][k][2] * inv, acc[j][k][3] * inv);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The insertion averages of k_contract_ins (Sec. II.C.3) on the matrix cores.  For one slot
// block (kMfSlots slots sharing (l, mode, spans)) and one position y of the
// displaced lines,
//   S[(r, c)][(k, kind)] = sum_m T_m^c(y - sh(r), r) O_m(y + ..., k, kind)
// (c: real or imaginary part of T) is a product of a (separation, part) x
// measurement matrix and a measurement x (slot, kind) matrix.  A tile
// (y, 8 separations) is one 16 x 16 FP64 accumulator and every MFMA step
// (v_mfma_f64_16x16x4) adds 4 measurements.  Lane L of a wave supplies
// A[i][q] and B[q][j] with i = j = L mod 16, q = L / 16, and holds
// D[L / 16 + 4 v][L mod 16], v = 0..3.  Row i stands for separation
// (i mod 4) + 4 (i / 8) of the tile and part (i / 4) mod 2, so that v = 0, 1
// are the real and imaginary part of separation L / 16 and v = 2, 3 of
// separation L / 16 + 4; column j is slot j / 2, kind j mod 2.
// Per chunk of mc measurements (a multiple of 4): the line's phases (16 bytes
// per work-item) and the O rows (4 bytes per work-item, so any axis and an
// odd row stride) are copied straight from memory into LDS while the
// previous chunk is summed; every T_m(x, r) of the chunk is then formed once
// into LDS; then the MFMA steps.  Measurements past the end add exact zeros
// (zero T values times finite O words).
// Work-group: one line, one slab, ins_pbw slot blocks, kMfThreads work-items;
// tiles (slot block, y, separation octet) in passes of 4 kMfTiles.
// ---------------------------------------------------------------------------
typedef double mf_d4 __attribute__((ext_vector_type(4)));

template <typename ot>
__global__ void __launch_bounds__(kMfThreads, 2) k_contract_mfma(
    const EnsDesc* __restrict__ ens, const int* __restrict__ bstart, int n_ens, const ObsDesc* __restrict__ obs,
    const int* __restrict__ rlist, const int* __restrict__ comps, const int* __restrict__ sblk,
    const double2* __restrict__ hist_c, const ot* __restrict__ hist_o, double2* __restrict__ avg_to, int n_meas,
    int n_blocks)
{
    // double-buffered chunks as separate LDS objects (no wait between the
    // copies into one and the reads of the other), T values of a chunk
    __shared__ double2 mph0[kMfPh], mph1[kMfPh];                  // phases [q][x]
    __shared__ __align__(16) unsigned mob0[kMfOb / 4], mob1[kMfOb / 4];  // O rows [q][row][y], padded
    __shared__ double mt[kMfT];                                    // T [q][x][r][part]
    __shared__ int rowoff[kMfRows];  // each O row's element offset within one (measurement, slab) block, -1: empty slot
    __shared__ int lr[kMfR];
    // XCD-aware order, as k_contract_ins
    const int bid = (int)(blockIdx.x & 7u) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
    if (bid >= n_blocks) return;
    const int e = find_ens_m(bstart, n_ens, bid);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int S = E.s_in, s = blockIdx.y;
    if (s >= S) return;
    const int id = blockIdx.z;
    const int dir = O.dirs[id];
    const int n3[3] = {E.nx, E.ny, E.nz};
    const int N = n3[dir];
    const int d1 = dir == 2 ? 0 : dir + 1, d2 = dir == 0 ? 2 : dir - 1;
    const int nsig = E.nsig, nlines = nsig / N;
    const int nr = O.n_r, nrt = (nr + 7) >> 3;
    const int nsb = O.n_pblocks, bpw = E.ins_pbw, nchunk = (nsb + bpw - 1) / bpw;
    const int local = bid - bstart[e];
    const int line = local / nchunk, chunk = local - line * nchunk;
    if (line >= nlines) return;  // uniform
    const int sb0 = chunk * bpw, nbw = min(bpw, nsb - sb0);
    const int nrows = nbw * 2 * kMfSlots;
    const int mc = E.ins_mc;
    constexpr int W = (int)sizeof(ot) / 4;  // 32-bit words per O element
    const int a1 = line % n3[d1], a2 = line / n3[d1];
    const int stride = dir == 0 ? 1 : (dir == 1 ? E.nx : E.nx * E.ny);
    auto site0 = [&](int o1, int o2) {
        int c[3];
        c[dir] = 0;
        c[d1] = ((a1 + o1) % n3[d1] + n3[d1]) % n3[d1];
        c[d2] = ((a2 + o2) % n3[d2] + n3[d2]) % n3[d2];
        return c[0] + E.nx * (c[1] + E.ny * c[2]);
    };
    const int base = site0(0, 0);
    const size_t mstride = (size_t)S * nsig;
    const size_t mstride_o = (size_t)S * 12 * nsig;
    const double2* hc = hist_c + E.hc_off + (size_t)s * nsig + base;
    const ot* ho = hist_o + E.ho_off + (size_t)s * 12 * nsig;
    const double inv = 1.0 / (double)n_meas;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = kMfThreads / 64;
    const bool vec = stride == 1 && (N * W) % 4 == 0 && (nsig * W) % 4 == 0 && (E.nx * W) % 4 == 0 &&
                     (mstride_o * W) % 4 == 0 && (reinterpret_cast<uintptr_t>(ho) & 15) == 0;
    const int rsd = vec ? N * W + 4 : (N + 1) * W;  // O row stride in LDS (words)
    const int qd = nrows * rsd;                     // words of one measurement's O rows in LDS
    for (int j = tid; j < nrows; j += kMfThreads) {
        const int bl = j / (2 * kMfSlots), rem = j - bl * 2 * kMfSlots, k = rem >> 1, kind = rem & 1;
        const int* B = sblk + kInsBlkInts * (sb0 + bl);
        int off = -1;
        if (k < B[3]) {
            const int* sl = B + 4 + 4 * k;  // probe, component index, p1, p2
            off = (2 * comp_orient(comps[sl[1]], dir) + kind) * nsig + site0(sl[2], sl[3]);
        }
        rowoff[j] = off;
    }
    for (int j = tid; j < nr; j += kMfThreads) lr[j] = rlist[j];
    // words of the O buffers that no copy writes (empty slots, row padding,
    // measurements past the end) stay finite: zero at the start, earlier
    // measurements' O values later
    for (int j = tid; j < kMfOb / 4; j += kMfThreads) {
        mob0[j] = 0u;
        mob1[j] = 0u;
    }
    // O rows of a chunk in units of U words: U = 4 (16-byte copies) where the
    // rows are contiguous and 16-byte aligned in memory (the x axis) and the
    // LDS row stride is N W + 4 words; else U = 1 with the odd stride
    // (N + 1) W, whose reads at one y fall in distinct banks.  Unit
    // u = (q nrows + row) (rsd / U) + c, of which the first N W / U of a row
    // carry data; each lane walks its units with a carry and keeps the
    // element offset q mstride_o of its measurement
    constexpr int VW = 4 / W;  // O elements per 16 bytes
    const int U = vec ? 4 : 1;
    const int nru = rsd / U, ndu = N * W / U, qu = nrows * nru;
    const int ostep = NW * 64;
    const int odq = ostep / qu, odr = ostep - odq * qu, odrow = odr / nru, odc = odr - odrow * nru;
    const int ou0 = wv * 64 + lane, oq0 = ou0 / qu, or0 = ou0 - oq0 * qu, orow0 = or0 / nru, oc0 = or0 - orow0 * nru;
    auto issue = [&](int m0, int mm, double2* php, unsigned* op) {
        for (int j = wv; j * 64 < mm * N; j += NW) {
            const int v = j * 64 + lane;
            if (v < mm * N) {
                const int q = v / N, x = v - q * N;
                __builtin_amdgcn_global_load_lds((const void*)(hc + (size_t)(m0 + q) * mstride + (size_t)x * stride),
                                                 (__attribute__((address_space(3))) void*)(php + j * 64), 16, 0, 0);
            }
        }
        const ot* hm = ho + (size_t)m0 * mstride_o;
        int q = oq0, row = orow0, c = oc0;
        size_t qoff = (size_t)oq0 * mstride_o;
        const size_t dqoff = (size_t)odq * mstride_o;
        for (int j = wv; j * 64 < mm * qu; j += NW) {
            if (q < mm && c < ndu) {
                const int off = rowoff[row];
                if (off >= 0) {
                    if (vec) {
                        __builtin_amdgcn_global_load_lds((const void*)(hm + qoff + off + c * VW),
                                                         (__attribute__((address_space(3))) void*)(op + j * 256), 16, 0,
                                                         0);
                    } else {
                        const int y = c / W, h = c - y * W;
                        const unsigned* src = reinterpret_cast<const unsigned*>(hm + qoff + off + (size_t)y * stride) + h;
                        __builtin_amdgcn_global_load_lds((const void*)src,
                                                         (__attribute__((address_space(3))) void*)(op + j * 64), 4, 0, 0);
                    }
                }
            }
            c += odc;
            if (c >= nru) {
                c -= nru;
                ++row;
            }
            row += odrow;
            if (row >= nrows) {
                row -= nrows;
                ++q;
                qoff += mstride_o;
            }
            q += odq;
            qoff += dqoff;
        }
    };
    // T_m(x, r) of a chunk, element f = (q N + x) nr + ir of [q][x][r] for
    // f = tid, tid + kMfThreads, ... (walked with a carry); zeros for the
    // measurements that pad the last MFMA step
    const int tqx = nr * N;
    const int tdq = kMfThreads / tqx, trm = kMfThreads - tdq * tqx, tdx = trm / nr, tdr = trm - tdx * nr;
    const int tq0 = tid / tqx, tr0 = tid - tq0 * tqx, tx0 = tr0 / nr, tir0 = tr0 - tx0 * nr;
    auto form_t = [&](int mm, const double2* ph) {
        const int mq = (mm + 3) & ~3;
        int q = tq0, x = tx0, ir = tir0;
        double2* tp = reinterpret_cast<double2*>(mt);
#pragma unroll 2
        for (int f = tid; f < mq * tqx; f += kMfThreads) {
            double2 t = make_double2(0.0, 0.0);
            if (q < mm) {
                int xb = x + lr[ir];
                xb -= xb >= N ? N : 0;
                const double2 a = ph[q * N + x], b = ph[q * N + xb];
                t = make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
            }
            tp[f] = t;
            ir += tdr;
            if (ir >= nr) {
                ir -= nr;
                ++x;
            }
            x += tdx;
            if (x >= N) {
                x -= N;
                ++q;
            }
            q += tdq;
        }
    };
    const int g16 = lane & 15, kq = lane >> 4;
    const int ntile = nbw * N * nrt, cap = NW * kMfTiles;
    const int nch = (n_meas + mc - 1) / mc;
    for (int tb = 0; tb < ntile; tb += cap) {
        const int t0 = tb + wv * kMfTiles;
        const int ntl = __builtin_amdgcn_readfirstlane(max(0, min(kMfTiles, ntile - t0)));  // uniform for the wave
        __syncthreads();  // row offsets and separations written; the previous pass done with every buffer
        // tile t = (bl N + y) nrt + rt: the wave's first by division, the next ones by a carry
        const int tbl0 = t0 / (N * nrt), trem0 = t0 - tbl0 * N * nrt, ty0 = trem0 / nrt, trt0 = trem0 - ty0 * nrt;
        auto next_tile = [&](int& bl, int& y, int& rt) {
            if (++rt == nrt) {
                rt = 0;
                if (++y == N) {
                    y = 0;
                    ++bl;
                }
            }
        };
        int a_off[kMfTiles], b_off[kMfTiles];
        int bl = tbl0, y = ty0, rt = trt0;
#pragma unroll
        for (int i = 0; i < kMfTiles; ++i) {
            if (i > 0 && i < ntl) next_tile(bl, y, rt);
            const int* B = sblk + kInsBlkInts * (sb0 + min(bl, nbw - 1));
            const int ir = min(rt * 8 + (g16 & 3) + 4 * (g16 >> 3), nr - 1), c = (g16 >> 2) & 1;
            const int r = lr[ir];
            const int sh = B[0] + (B[1] ? (B[2] ? (r - 1) / 2 : r / 2) : 0);
            int x = (y - sh) % N;
            x += x < 0 ? N : 0;
            a_off[i] = (x * nr + ir) * 2 + c;
            b_off[i] = (min(bl, nbw - 1) * 2 * kMfSlots + g16) * rsd + y * W;
        }
        mf_d4 acc[kMfTiles];
#pragma unroll
        for (int i = 0; i < kMfTiles; ++i) acc[i] = mf_d4{0.0, 0.0, 0.0, 0.0};
        auto mfma_chunk = [&](int mm, const unsigned* op) {
            // the T values of measurements past mm are zero and every O word is finite
            for (int st = 0; st < mm; st += 4) {
                const int q = st + kq;
                const int qa = q * N * nr * 2, qb = q * qd;
                // operands of 4 tiles at a time, then their 4 steps
#pragma unroll
                for (int i0 = 0; i0 < kMfTiles; i0 += 4) {
                    double av[4], bv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + u;
                        if (i < ntl) {
                            av[u] = mt[qa + a_off[i]];
                            if constexpr (W == 1) {
                                bv[u] = (double)__uint_as_float(op[qb + b_off[i]]);
                            } else {
                                bv[u] = *reinterpret_cast<const double*>(op + qb + b_off[i]);
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (i0 + u < ntl)
                            acc[i0 + u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc[i0 + u], 0, 0, 0);
                }
            }
        };
        // chunk ci lives in buffers ci mod 2: before its T values are formed,
        // this wave's copies into it have landed (vmcnt 0) and the barrier
        // makes every wave's visible and ends the sums over chunk ci - 1,
        // whose buffers the copies of chunk ci + 1 then overwrite; the second
        // barrier publishes the T values
        auto step = [&](int ci, const double2* ph, const unsigned* op, double2* nph, unsigned* nop) {
            const int mm = min(mc, n_meas - ci * mc);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
            __syncthreads();
            if (ci + 1 < nch) issue((ci + 1) * mc, min(mc, n_meas - (ci + 1) * mc), nph, nop);
            form_t(mm, ph);
            __syncthreads();
            mfma_chunk(mm, op);
        };
        issue(0, min(mc, n_meas), mph0, mob0);
        for (int ci = 0; ci < nch; ci += 2) {
            step(ci, mph0, mob0, mph1, mob1);
            if (ci + 1 >= nch) break;
            step(ci + 1, mph1, mob1, mph0, mob0);
        }
        bl = tbl0;
        y = ty0;
        rt = trt0;
#pragma unroll
        for (int i = 0; i < kMfTiles; ++i) {
            if (i >= ntl) continue;
            if (i > 0) next_tile(bl, y, rt);
            const int* B = sblk + kInsBlkInts * (sb0 + bl);
            const int k = g16 >> 1, kind = g16 & 1;
            if (k >= B[3]) continue;
            const int p = B[4 + 4 * k], ic = B[5 + 4 * k];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int ir = rt * 8 + kq + 4 * h;
                if (ir >= nr) continue;
                const int r = lr[ir];
                const int sh = B[0] + (B[1] ? (B[2] ? (r - 1) / 2 : r / 2) : 0);
                int x = (y - sh) % N;
                x += x < 0 ? N : 0;
                const size_t kk = ((((size_t)id * nr + ir) * O.n_probe + p) * O.n_comp + ic) * 2 + kind;
                avg_to[E.ato_off + (kk * S + s) * nsig + base + (size_t)x * stride] =
                    make_double2(acc[i][2 * h] * inv, acc[i][2 * h + 1] * inv);
            }
        }
    }
}

hipError_t launch_contract(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, int block,
                           size_t lds_bytes, const ObsDesc* d_obs, const int* d_r, const double2* hist_c,
                           double2* avg_t, int n_meas, int max_slabs, int n_dirs, hipStream_t st)
{
    hipLaunchKernelGGL(k_contract, dim3(total_blocks, max_slabs, n_dirs), dim3(block), lds_bytes, st, d_ens, d_bstart,
                       n_ens, d_obs, d_r, hist_c, avg_t, n_meas);
    return hipGetLastError();
}

hipError_t launch_contract_ins(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, int block,
                               size_t lds_bytes, const ObsDesc* d_obs, const int* d_r, const int* d_comp,
                               const int* d_sblk, int slots_per_block, const double2* hist_c, const void* hist_o,
                               double2* avg_to, int n_meas, int precision, int max_slabs, int n_dirs, int line_len,
                               hipStream_t st)
{
    if (total_blocks <= 0) return hipSuccess;
    const dim3 g((total_blocks + 7) / 8 * 8, max_slabs, n_dirs), b(block);
#define U1ML_INS(OT, KR, KS)                                                                                          \
    do {                                                                                                              \
        if (line_len == 24)                                                                                           \
            hipLaunchKernelGGL((k_contract_ins<OT, KR, KS, 24>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs,   \
                               d_r, d_comp, d_sblk, hist_c, (const OT*)hist_o, avg_to, n_meas, total_blocks);         \
        else                                                                                                          \
            hipLaunchKernelGGL((k_contract_ins<OT, KR, KS, 0>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs,    \
                               d_r, d_comp, d_sblk, hist_c, (const OT*)hist_o, avg_to, n_meas, total_blocks);         \
    } while (0)
    if (slots_per_block == kMfSlots) {
        if (precision == 0)
            hipLaunchKernelGGL(k_contract_mfma<double>, g, dim3(kMfThreads), 0, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               d_comp, d_sblk, hist_c, (const double*)hist_o, avg_to, n_meas, total_blocks);
        else
            hipLaunchKernelGGL(k_contract_mfma<float>, g, dim3(kMfThreads), 0, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               d_comp, d_sblk, hist_c, (const float*)hist_o, avg_to, n_meas, total_blocks);
        return hipGetLastError();
    }
    if (precision == 0) {
        switch (slots_per_block) {
        case 9: U1ML_INS(double, ins_kr(9), 9); break;
        case 6: U1ML_INS(double, ins_kr(6), 6); break;
        case 3: U1ML_INS(double, ins_kr(3), 3); break;
        default: U1ML_INS(double, ins_kr(1), 1); break;
        }
    } else {
        switch (slots_per_block) {
        case 9: U1ML_INS(float, ins_kr(9), 9); break;
        case 6: U1ML_INS(float, ins_kr(6), 6); break;
        case 3: U1ML_INS(float, ins_kr(3), 3); break;
        default: U1ML_INS(float, ins_kr(1), 1); break;
        }
    }
#undef U1ML_INS
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Two-level combine, one work-item per (ensemble, axis, r, thick slab S, x):
//   out_t(S)  += prod_j [T](S q + j)
//   out_to(S) += sum_j [TO](S q + j) prod_{j' != j} [T](S q + j')
// ---------------------------------------------------------------------------
__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

__global__ void __launch_bounds__(256) k_combine(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                 int n_ens, const ObsDesc* __restrict__ obs,
                                                 const double2* __restrict__ avg_t, const double2* __restrict__ avg_to,
                                                 double2* __restrict__ out_t, double2* __restrict__ out_to, int q)
{
    const int bid = blockIdx.x;
    const int e = find_ens_m(bstart, n_ens, bid);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int nsig = E.nsig, Si = E.s_in, So = E.s_out;
    const long long item = (long long)(bid - bstart[e]) * blockDim.x + threadIdx.x;
    if (item >= (long long)O.n_dirs * O.n_r * So * nsig) return;
    const int xs = (int)(item % nsig);
    long long rest = item / nsig;
    const int S = (int)(rest % So);
    const long long idr = rest / So;  // id * n_r + ir
    double2 A[8];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        A[j] = j < q ? avg_t[E.at_off + ((size_t)idr * Si + S * q + j) * nsig + xs] : make_double2(1.0, 0.0);
    double2 T4 = make_double2(1.0, 0.0);
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < q) T4 = cmul(T4, A[j]);
    double2* ot = out_t + E.ot_off + ((size_t)idr * So + S) * nsig + xs;
    *ot = make_double2(ot->x + T4.x, ot->y + T4.y);
    if (!avg_to) return;  // spectral form: no per-site insertion averages
    const long long n_to = (long long)O.n_probe * O.n_comp * 2;
    for (long long k = 0; k < n_to; ++k) {
        const size_t row = (size_t)idr * n_to + k;
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < q) {
                double2 term = avg_to[E.ato_off + (row * Si + S * q + j) * nsig + xs];
#pragma unroll
                for (int j2 = 0; j2 < 8; ++j2)
                    if (j2 < q && j2 != j) term = cmul(term, A[j2]);
                acc.x += term.x;
                acc.y += term.y;
            }
        }
        double2* oo = out_to + E.oto_off + (row * So + S) * nsig + xs;
        *oo = make_double2(oo->x + acc.x, oo->y + acc.y);
    }
}

hipError_t launch_combine(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, const ObsDesc* d_obs,
                          const double2* avg_t, const double2* avg_to, double2* out_t, double2* out_to, int q,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_combine, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, avg_t, avg_to,
                       out_t, out_to, q);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Slab products and sums over sites (Sec. II.C.2-3).  The products over many
// slabs of averages of modulus below one can leave the range of FP64, so they
// run as scaled complex numbers, and both sums are taken relative to 2^E(r),
// E(r) the largest binary exponent of the per-site correlator products of
// separation r over the charge axes and sites (0 if they all vanish).  The
// record holds the mantissas and E(r); values in range are unchanged bit for
// bit by the scaling.
//
// Three launches, each over the work-group table of (e, r, probe group, site
// chunk):
//   k_prod_exp:      the largest exponent of each chunk (probe group 0 only),
//                    kept in the first slot of the chunk's partials;
//   k_prod_exp_final: E(r) of each (e, r) from its chunks, written to the
//                    configuration's record (where the products and the
//                    spectral weights read it);
//   k_product:       every thread walks the chunk's (axis, x) items in a fixed
//                    stride, forms P(x) = prod_S A(S) and W_S(x) =
//                    prod_{S' != S} A(S'), and adds P 2^-E (correlator, probe 0
//                    only) and sum_S B(S) W_S 2^-E (insertions) to
//                    double-double accumulators; a fixed-order tree reduces the
//                    work-group into part[wg][26][hi, lo];
//   k_product_final: the chunks of each (e, r, probe) in chunk order.
// src_t  = A * scale_t, src_to = B * scale_t (scale_t = 1 or 1/n_outer).
// ---------------------------------------------------------------------------
struct ProdItem {
    int e, ir, p, ch;
};

__device__ inline bool prod_item(const int* __restrict__ bstart, int n_ens, const EnsDesc* __restrict__ ens,
                                 int n_r, int n_pgroups, ProdItem* o)
{
    o->e = find_ens_m(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[o->e];
    const int local = blockIdx.x - bstart[o->e];
    o->ch = local % E.prod_nch;
    o->p = (local / E.prod_nch) % n_pgroups;
    o->ir = local / (E.prod_nch * n_pgroups);
    return o->ir < n_r;  // the work-group table holds n_r * n_pgroups * prod_nch per ensemble (uniform)
}

// the current configuration's record of ensemble E
template <typename T>
__device__ inline T* record_of(const EnsDesc& E, const ObsDesc& O, T* results, const int* ring)
{
    return results + ((size_t)(*ring) * O.n_ens_total + E.res_index) * O.n_doubles_per_config;
}

__device__ inline sc slab_product(const double2* __restrict__ row, int S, int nsig, int skip, double scale_t)
{
    sc P{1.0, 0.0, 0};
    for (int s = 0; s < S; ++s) {
        if (s == skip) continue;
        double2 a = row[(size_t)s * nsig];
        a.x *= scale_t;
        a.y *= scale_t;
        P = sc_mul(P, a);
    }
    return P;
}

__global__ void __launch_bounds__(256) k_prod_exp(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                  int n_ens, const ObsDesc* __restrict__ obs, int n_pgroups,
                                                  const double2* __restrict__ src_t, int use_outer, double scale_t,
                                                  double* __restrict__ part)
{
    const ObsDesc& O = *obs;
    ProdItem I;
    if (!prod_item(bstart, n_ens, ens, O.n_r, n_pgroups, &I) || I.p != 0) return;
    const EnsDesc& E = ens[I.e];
    const int nsig = E.nsig;
    const int S = use_outer ? E.s_out : E.s_in;
    const long long t_off = use_outer ? E.ot_off : E.at_off;
    const int n_items = O.n_dirs * nsig;
    const int it_end = min(n_items, (I.ch + 1) * kProdChunk);
    int emax = kNoExp;
    for (int it = I.ch * kProdChunk + (int)threadIdx.x; it < it_end; it += blockDim.x) {
        const int id = it / nsig, xs = it - id * nsig;
        const double2* row = src_t + t_off + ((size_t)id * O.n_r + I.ir) * S * nsig + xs;
        emax = max(emax, sc_exp(slab_product(row, S, nsig, -1, scale_t)));
    }
    __shared__ int sh[256];
    sh[threadIdx.x] = emax;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * kProdQ * 2] = (double)sh[0];
}

// one work-item per (e, r)
__global__ void __launch_bounds__(64) k_prod_exp_final(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                       int n_ens, const ObsDesc* __restrict__ obs, int n_pgroups,
                                                       const double* __restrict__ part, double* __restrict__ results,
                                                       const int* __restrict__ ring)
{
    const ObsDesc& O = *obs;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ens * O.n_r) return;
    const int e = i / O.n_r, ir = i % O.n_r;
    const EnsDesc& E = ens[e];
    const int b0 = bstart[e] + ir * n_pgroups * E.prod_nch;  // probe group 0
    int emax = kNoExp;
    for (int c = 0; c < E.prod_nch; ++c) emax = max(emax, (int)part[(size_t)(b0 + c) * kProdQ * 2]);
    record_of(E, O, results, ring)[O.n_doubles_per_config - O.n_r + ir] = emax == kNoExp ? 0.0 : (double)emax;
}

__global__ void __launch_bounds__(256) k_product(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                 int n_ens, const ObsDesc* __restrict__ obs, int n_pgroups,
                                                 const double2* __restrict__ src_t, const double2* __restrict__ src_to,
                                                 int use_outer, double scale_t, double* __restrict__ part,
                                                 const double* __restrict__ results, const int* __restrict__ ring)
{
    const ObsDesc& O = *obs;
    const int n_r = O.n_r;
    ProdItem I;
    if (!prod_item(bstart, n_ens, ens, n_r, n_pgroups, &I)) return;
    const EnsDesc& E = ens[I.e];
    const int ch = I.ch, p = I.p, ir = I.ir;
    const int nsig = E.nsig;
    const int S = use_outer ? E.s_out : E.s_in;
    const long long t_off = use_outer ? E.ot_off : E.at_off;
    const long long to_off = use_outer ? E.oto_off : E.ato_off;
    const int nc = O.n_comp;
    const bool has_probe = O.n_probe > 0 && src_to != nullptr;  // null: insertions come from the spectral form
    const int Er = (int)record_of(E, O, results, ring)[O.n_doubles_per_config - n_r + ir];
    dd cre{0, 0}, cim{0, 0};
    dd ore[12], oim[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        ore[k] = dd{0, 0};
        oim[k] = dd{0, 0};
    }
    const int n_items = O.n_dirs * nsig;
    const int it_end = min(n_items, (ch + 1) * kProdChunk);
    for (int it = ch * kProdChunk + (int)threadIdx.x; it < it_end; it += blockDim.x) {
        const int id = it / nsig, xs = it - id * nsig;
        const double2* row = src_t + t_off + ((size_t)id * n_r + ir) * S * nsig + xs;
        if (p == 0) {
            const double2 v = sc_rel(slab_product(row, S, nsig, -1, scale_t), Er);
            cre = dd_add(cre, v.x);
            cim = dd_add(cim, v.y);
        }
        if (!has_probe) continue;
        for (int s = 0; s < S; ++s) {
            const sc W = slab_product(row, S, nsig, s, scale_t);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                if (k < 2 * nc) {
                    const size_t krow = ((((size_t)id * n_r + ir) * O.n_probe + p) * nc) * 2 + k;
                    double2 b = src_to[to_off + (krow * S + s) * nsig + xs];
                    b.x *= scale_t;
                    b.y *= scale_t;
                    const double2 v = sc_rel(sc_mul(W, b), Er);
                    ore[k] = dd_add(ore[k], v.x);
                    oim[k] = dd_add(oim[k], v.y);
                }
            }
        }
    }
    __shared__ double shh[256], shl[256];
    auto reduce = [&](dd v) -> dd {
        shh[threadIdx.x] = v.hi;
        shl[threadIdx.x] = v.lo;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                const dd a = dd_add(dd{shh[threadIdx.x], shl[threadIdx.x]},
                                    dd{shh[threadIdx.x + w], shl[threadIdx.x + w]});
                shh[threadIdx.x] = a.hi;
                shl[threadIdx.x] = a.lo;
            }
            __syncthreads();
        }
        const dd r{shh[0], shl[0]};
        __syncthreads();
        return r;
    };
    double* out = part + (size_t)blockIdx.x * kProdQ * 2;
    auto put = [&](int q, dd v) {
        if (threadIdx.x == 0) {
            out[2 * q] = v.hi;
            out[2 * q + 1] = v.lo;
        }
    };
    if (p == 0) {
        put(0, reduce(cre));
        put(1, reduce(cim));
    }
    if (has_probe) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            if (k < 2 * nc) {  // uniform
                put(2 + 2 * k, reduce(ore[k]));
                put(3 + 2 * k, reduce(oim[k]));
            }
        }
    }
}

// One work-item per (e, r, probe group, quantity): the chunk partials in
// chunk order, normalised and written to the configuration's result row.
__global__ void __launch_bounds__(64) k_product_final(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                      int n_ens, const ObsDesc* __restrict__ obs, int n_pgroups,
                                                      const double* __restrict__ part, double* __restrict__ results,
                                                      const int* __restrict__ ring, int with_ins)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const ObsDesc& O = *obs;
    const int n_r = O.n_r;
    if (i >= n_ens * n_r * n_pgroups * kProdQ) return;
    const int q = i % kProdQ;
    const int p = (i / kProdQ) % n_pgroups;
    const int ir = (i / (kProdQ * n_pgroups)) % n_r;
    const int e = i / (kProdQ * n_pgroups * n_r);
    const EnsDesc& E = ens[e];
    const int nc = O.n_comp;
    if (q < 2 && p != 0) return;
    if (q >= 2 && (!with_ins || O.n_probe == 0 || q - 2 >= 4 * nc)) return;
    const int b0 = bstart[e] + (ir * n_pgroups + p) * E.prod_nch;
    // chunks added in order; the loads of eight chunks are issued before their additions
    dd a{0.0, 0.0};
    const double* src = part + ((size_t)b0 * kProdQ + q) * 2;
    constexpr size_t cs = (size_t)kProdQ * 2;
    int c = 0;
    for (; c + 8 <= E.prod_nch; c += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = make_double2(src[(c + u) * cs], src[(c + u) * cs + 1]);
#pragma unroll
        for (int u = 0; u < 8; ++u) a = dd_add(a, dd{v[u].x, v[u].y});
    }
    for (; c < E.prod_nch; ++c) a = dd_add(a, dd{src[c * cs], src[c * cs + 1]});
    double* out = record_of(E, O, results, ring);
    const double nC = 1.0 / ((double)E.nsig * O.n_dirs);
    if (q < 2) {
        out[2 * ir + q] = (a.hi + a.lo) * nC;
    } else {
        const int k = (q - 2) >> 1, im = (q - 2) & 1;
        const long long idx = (((long long)ir * O.n_probe + p) * nc) * 2 + k;
        out[2ll * n_r + 2 * idx + im] = (a.hi + a.lo) * (nC / (double)E.nt);
    }
}

hipError_t launch_prod_exp(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks,
                           const ObsDesc* d_obs, int n_r, int n_pgroups, const double2* src_t, int use_outer,
                           double scale, double* part, double* results, const int* d_ring, hipStream_t st)
{
    hipLaunchKernelGGL(k_prod_exp, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, n_pgroups,
                       src_t, use_outer, scale, part);
    const int ne = n_ens * n_r;
    hipLaunchKernelGGL(k_prod_exp_final, dim3((ne + 63) / 64), dim3(64), 0, st, d_ens, d_bstart, n_ens, d_obs,
                       n_pgroups, part, results, d_ring);
    return hipGetLastError();
}

hipError_t launch_product(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks,
                          const ObsDesc* d_obs, int n_r, int n_pgroups, const double2* src_t, const double2* src_to,
                          int use_outer, double scale, double* part, double* results, const int* d_ring,
                          hipStream_t st)
{
    hipError_t e = launch_prod_exp(d_ens, d_bstart, n_ens, total_blocks, d_obs, n_r, n_pgroups, src_t, use_outer,
                                   scale, part, results, d_ring, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_product, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, n_pgroups,
                       src_t, src_to, use_outer, scale, part, results, d_ring);
    const int nq = n_ens * n_r * n_pgroups * kProdQ;
    hipLaunchKernelGGL(k_product_final, dim3((nq + 63) / 64), dim3(64), 0, st, d_ens, d_bstart, n_ens, d_obs, n_pgroups,
                       part, results, d_ring, src_to != nullptr ? 1 : 0);
    return hipGetLastError();
}

// vacuum <O_sq>, <O_lin> per orientation: the running block partials of the
// configuration summed in a fixed-order double-double tree, divided by
// (measurements * V).  Block (e, k) reduces quantity k of ensemble e.
__global__ void __launch_bounds__(256) k_vac_final(const EnsDesc* __restrict__ ens, int n_ens,
                                                   const ObsDesc* __restrict__ obs, const double* __restrict__ vac_part,
                                                   int n_meas, double* __restrict__ results,
                                                   const int* __restrict__ ring)
{
    const int e = blockIdx.x / 12, k = blockIdx.x % 12;
    const EnsDesc& E = ens[e];
    // partials i = tid, tid + 256, ... added in order; the loads of eight are
    // issued before their additions
    dd a{0.0, 0.0};
    const double* vp = vac_part + E.vac_part_off + 2 * k;
    const int nb = E.n_vac_blocks;
    int i = threadIdx.x;
    for (; i + 7 * (int)blockDim.x < nb; i += 8 * blockDim.x) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double* p = vp + (size_t)(i + u * blockDim.x) * 24;
            v[u] = make_double2(p[0], p[1]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) a = dd_add(a, dd{v[u].x, v[u].y});
    }
    for (; i < nb; i += blockDim.x) {
        const double* p = vp + (size_t)i * 24;
        a = dd_add(a, dd{p[0], p[1]});
    }
    __shared__ double shh[256], shl[256];
    shh[threadIdx.x] = a.hi;
    shl[threadIdx.x] = a.lo;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const dd b = dd_add(dd{shh[threadIdx.x], shl[threadIdx.x]}, dd{shh[threadIdx.x + w], shl[threadIdx.x + w]});
            shh[threadIdx.x] = b.hi;
            shl[threadIdx.x] = b.lo;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const ObsDesc& O = *obs;
        const long long base_v = 2ll * O.n_r + 4ll * O.n_r * O.n_probe * O.n_comp;
        double* out = results + ((size_t)(*ring) * O.n_ens_total + E.res_index) * O.n_doubles_per_config;
        // accumulator order is (o, kind); output order is sq[6] then lin[6]
        const int o = k >> 1, kind = k & 1;
        out[base_v + kind * 6 + o] = (shh[0] + shl[0]) / ((double)n_meas * 2.0 * (double)E.vh);
    }
}

hipError_t launch_vac_final(const EnsDesc* d_ens, int n_ens, const ObsDesc* d_obs, const double* vac_part, int n_meas,
                            double* results, const int* d_ring, hipStream_t st)
{
    hipLaunchKernelGGL(k_vac_final, dim3(n_ens * 12), dim3(256), 0, st, d_ens, n_ens, d_obs, vac_part, n_meas, results,
                       d_ring);
    return hipGetLastError();
}

__global__ void k_ring_advance(int* ring)
{
    if (threadIdx.x == 0) ring[0] += 1;
}

hipError_t launch_ring_advance(int* d_ring, hipStream_t st)
{
    hipLaunchKernelGGL(k_ring_advance, dim3(1), dim3(64), 0, st, d_ring);
    return hipGetLastError();
}

}  // namespace u1ml
