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
#include "device_common.hpp"
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

// scaled complex: value = (re + i im) * 2^ex, max(|re|,|im|) in [1, 2) or 0
struct sc {
    double re, im;
    int ex;
};

__device__ inline sc sc_norm(double re, double im, int ex)
{
    const double m = fmax(fabs(re), fabs(im));
    if (m == 0.0 || !isfinite(m)) return sc{re, im, 0};
    const int k = ilogb(m);
    return sc{ldexp(re, -k), ldexp(im, -k), ex + k};
}

__device__ inline sc sc_mul(sc a, double2 b)
{
    return sc_norm(a.re * b.x - a.im * b.y, a.re * b.y + a.im * b.x, a.ex);
}

__device__ inline sc sc_mul(sc a, sc b)
{
    return sc_norm(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re, a.ex + b.ex);
}

__device__ inline double2 sc_val(sc a) { return make_double2(ldexp(a.re, a.ex), ldexp(a.im, a.ex)); }

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
//   hist_o[m_in][s][2o+k][x] = sum_{t in s} O_k(P_o(x, t)); k = 0: 2 beta (1 - cos),
//                              k = 1: sqrt(beta) sin, orientations o = P_xt, P_yt,
//                              P_zt, P_yz, P_zx, P_xy
//   vac_part[m][block][2o+k] = block sum of O_k over every plaquette (vacuum <O>)
// m_in indexes the measurement inside the innermost level, m the measurement
// inside the configuration.
// ---------------------------------------------------------------------------
template <typename real>
__device__ inline void plaq_O(real th, double beta, double sqrt_beta, double* osq, double* olin);

template <>
__device__ inline void plaq_O<double>(double th, double beta, double sqrt_beta, double* osq, double* olin)
{
    double s, c;
    sincos(th, &s, &c);
    *osq = 2.0 * beta * (1.0 - c);
    *olin = sqrt_beta * s;
}

template <>
__device__ inline void plaq_O<float>(float th, double beta, double sqrt_beta, double* osq, double* olin)
{
    // 1 - cos(th) = 2 sin^2(th / 2), free of cancellation in FP32
    const float rev = th * 0.159154943f;
    const float sh = __builtin_amdgcn_sinf(0.5f * rev);
    const float s = __builtin_amdgcn_sinf(rev);
    *osq = 4.0 * beta * (double)(sh * sh);
    *olin = sqrt_beta * (double)s;
}

// Sum of 12 per-thread doubles over a 256-thread block in a fixed order:
// through LDS, each wave then reduces three of the quantities.
__device__ inline void block_sum12(const double* v, double* out)
{
    __shared__ double red[12][256];
#pragma unroll
    for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        const int k = 3 * wave + kk;
        double a = red[k][lane] + red[k][lane + 64] + red[k][lane + 128] + red[k][lane + 192];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        if (lane == 0) out[k] = a;
    }
}

template <typename real>
__global__ void __launch_bounds__(256) k_measure(const EnsDesc* __restrict__ ens, const int2* __restrict__ bmap,
                                                 const real* __restrict__ links, double2* __restrict__ hist_c,
                                                 real* __restrict__ hist_o, double* __restrict__ vac_part, int m_in,
                                                 int m, int tau, int store_o)
{
    const int2 be = bmap[blockIdx.x];
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
        const int s = item / nsig;
        const int xs = item - s * nsig;
        const int yz = xs / E.nx;
        const int x = xs - yz * E.nx;
        const int z = yz / E.ny;
        const int y = yz - z * E.ny;
        double Th = 0.0;
        double os[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) os[k] = 0.0;
        Site c{x, y, z, s * tau, g.sy * yz + g.st * (s * tau)};
        for (int k = 0; k < tau; ++k) {
            const unsigned p = (unsigned)((x + y + z + c.t) & 1), q = p ^ 1u;
            const Site cx = mv<0, +1>(c, g), cy = mv<1, +1>(c, g), cz = mv<2, +1>(c, g), ct = mv<3, +1>(c, g);
            auto L = [&](unsigned dir, unsigned par, const Site& st) {
                return ldo(lb, ((dir * 2u + par) * vh + hidx(st)) * w);
            };
            const real ux = L(0, p, c), uy = L(1, p, c), uz = L(2, p, c), ut = L(3, p, c);
            const real tx_x = L(3, q, cx), tx_y = L(3, q, cy), tx_z = L(3, q, cz);
            const real xt = L(0, q, ct), yt = L(1, q, ct), zt = L(2, q, ct);
            const real zy = L(2, q, cy), yz_ = L(1, q, cz);
            const real xz = L(0, q, cz), zx = L(2, q, cx);
            const real yx = L(1, q, cx), xy = L(0, q, cy);
            Th += (double)ut;
            real th[6];
            th[0] = ux + tx_x - xt - ut;  // P_xt
            th[1] = uy + tx_y - yt - ut;  // P_yt
            th[2] = uz + tx_z - zt - ut;  // P_zt
            th[3] = uy + zy - yz_ - uz;   // P_yz
            th[4] = uz + xz - zx - ux;    // P_zx
            th[5] = ux + yx - xy - uy;    // P_xy
#pragma unroll
            for (int o = 0; o < 6; ++o) {
                double a, b;
                plaq_O<real>(th[o], E.beta, E.sqrt_beta, &a, &b);
                os[2 * o] += a;
                os[2 * o + 1] += b;
            }
            c = ct;
        }
        double sn, cs;
        sincos(Th, &sn, &cs);
        hist_c[E.hc_off + ((size_t)m_in * S + s) * nsig + xs] = make_double2(cs, sn);
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
    block_sum12(vac, vac_part + E.vac_part_off + ((size_t)m * E.n_vac_blocks + be.y) * 12);
}

hipError_t launch_measure(const EnsDesc* d_ens, const int2* d_bmap, int total_blocks, int precision, const void* links,
                          double2* hist_c, void* hist_o, double* vac_part, int m_in, int m, int tau, int store_o,
                          hipStream_t st)
{
    if (precision == 0)
        hipLaunchKernelGGL(k_measure<double>, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bmap,
                           (const double*)links, hist_c, (double*)hist_o, vac_part, m_in, m, tau, store_o);
    else
        hipLaunchKernelGGL(k_measure<float>, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bmap,
                           (const float*)links, hist_c, (float*)hist_o, vac_part, m_in, m, tau, store_o);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inner-level contraction: one work-item per (ensemble, axis, r, slab s, x).
//   [T](s,x,r)  = 1/n sum_m conj(c_m(s,x)) c_m(s,x+r mu)
//   [TO](s,x,r,p,c,k) = 1/n sum_m T_m(s,x,r) Osum_m(s, x0(x,r,p,c), o(c,mu), k)
// ---------------------------------------------------------------------------
__device__ inline int shift_site(int x, int y, int z, int dir, int d, int nx, int ny, int nz)
{
    int c[3] = {x, y, z};
    const int n[3] = {nx, ny, nz};
    int v = (c[dir] + d) % n[dir];
    if (v < 0) v += n[dir];
    c[dir] = v;
    return c[0] + nx * (c[1] + ny * c[2]);
}

__device__ inline int probe_site(int x, int y, int z, int dir, int l, int p1, int p2, int nx, int ny, int nz)
{
    const int n[3] = {nx, ny, nz};
    int c[3] = {x, y, z};
    const int d1 = (dir + 1) % 3, d2 = (dir + 2) % 3;
    c[dir] = ((c[dir] + l) % n[dir] + n[dir]) % n[dir];
    c[d1] = ((c[d1] + p1) % n[d1] + n[d1]) % n[d1];
    c[d2] = ((c[d2] + p2) % n[d2] + n[d2]) % n[d2];
    return c[0] + nx * (c[1] + ny * c[2]);
}

template <typename ot>
__global__ void __launch_bounds__(256) k_contract(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                  int n_ens, const ObsDesc* __restrict__ obs,
                                                  const int* __restrict__ rlist, const int* __restrict__ probes,
                                                  const int* __restrict__ comps, const double2* __restrict__ hist_c,
                                                  const ot* __restrict__ hist_o, double2* __restrict__ avg_t,
                                                  double2* __restrict__ avg_to, int n_meas)
{
    const int bid = blockIdx.x;
    const int e = find_ens_m(bstart, n_ens, bid);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int nsig = E.nsig, S = E.s_in;
    // grid: x = (64 consecutive sites, then r, then the 64-site chunk) of one
    // ensemble, y = slab, z = charge axis; slab and axis are uniform per block,
    // so the history rows are addressed from scalar bases.  A block covers
    // several r for the same sites, so the shifted reads overlap in L1.
    const int s = blockIdx.y;
    const int id = blockIdx.z;
    if (s >= S) return;
    const int nchunk = (nsig + 63) / 64;
    const int item = (bid - bstart[e]) * (int)blockDim.x + (int)threadIdx.x;
    if (item >= nchunk * O.n_r * 64) return;
    const int lane = item & 63;
    const int rest = item >> 6;
    const int ir = rest % O.n_r;
    const int chunk = rest / O.n_r;
    const int xs = chunk * 64 + lane;
    if (xs >= nsig) return;
    const int dir = O.dirs[id];
    const int r = rlist[ir];
    const int x = xs % E.nx, y = (xs / E.nx) % E.ny, z = xs / (E.nx * E.ny);
    const int xr = shift_site(x, y, z, dir, r, E.nx, E.ny, E.nz);
    const size_t mstride = (size_t)S * nsig;
    const double2* hc = hist_c + E.hc_off + (size_t)s * nsig;
    const double inv = 1.0 / (double)n_meas;

    double tre = 0.0, tim = 0.0;
    for (int m = 0; m < n_meas; ++m) {
        const double2 a = hc[m * mstride + xs];
        const double2 b = hc[m * mstride + xr];
        tre += a.x * b.x + a.y * b.y;
        tim += a.x * b.y - a.y * b.x;
    }
    avg_t[E.at_off + (((size_t)id * O.n_r + ir) * S + s) * nsig + xs] = make_double2(tre * inv, tim * inv);

    // insertions: probes in chunks of 2, every component and both kinds;
    // per measurement, T is formed once and the chunk's 24 slab sums are read
    const int nc = O.n_comp;
    constexpr int PC = 2;
    for (int p0 = 0; p0 < O.n_probe; p0 += PC) {
        unsigned off[PC][6];  // element offset (orientation row + site) of each (probe, component)
#pragma unroll
        for (int pp = 0; pp < PC; ++pp) {
            const int p = p0 + pp < O.n_probe ? p0 + pp : p0;
            const int l = probes[4 * p], p1 = probes[4 * p + 1], p2 = probes[4 * p + 2], mode = probes[4 * p + 3];
            const int y_span = probe_site(x, y, z, dir, l + (mode ? (r - 1) / 2 : 0), p1, p2, E.nx, E.ny, E.nz);
            const int y_orth = probe_site(x, y, z, dir, l + (mode ? r / 2 : 0), p1, p2, E.nx, E.ny, E.nz);
#pragma unroll
            for (int ic = 0; ic < 6; ++ic) {
                const int c = ic < nc ? comps[ic] : 0;
                off[pp][ic] = (unsigned)(2 * comp_orient(c, dir)) * (unsigned)nsig +
                              (unsigned)(comp_spans_axis(c) ? y_span : y_orth);
            }
        }
        double acc[PC][6][4];
#pragma unroll
        for (int pp = 0; pp < PC; ++pp)
#pragma unroll
            for (int ic = 0; ic < 6; ++ic)
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[pp][ic][k] = 0.0;
        for (int m = 0; m < n_meas; ++m) {
            const double2 a = hc[m * mstride + xs];
            const double2 b = hc[m * mstride + xr];
            const ot* ho = hist_o + E.ho_off + ((size_t)m * S + s) * 12 * nsig;  // uniform
            double osq[PC][6], olin[PC][6];
#pragma unroll
            for (int pp = 0; pp < PC; ++pp)
#pragma unroll
                for (int ic = 0; ic < 6; ++ic) {
                    osq[pp][ic] = ic < nc ? (double)ldo(ho, off[pp][ic] * (unsigned)sizeof(ot)) : 0.0;
                    olin[pp][ic] = ic < nc ? (double)ldo(ho, (off[pp][ic] + nsig) * (unsigned)sizeof(ot)) : 0.0;
                }
            const double Tr = a.x * b.x + a.y * b.y;
            const double Ti = a.x * b.y - a.y * b.x;
#pragma unroll
            for (int pp = 0; pp < PC; ++pp)
#pragma unroll
                for (int ic = 0; ic < 6; ++ic) {
                    acc[pp][ic][0] += Tr * osq[pp][ic];
                    acc[pp][ic][1] += Ti * osq[pp][ic];
                    acc[pp][ic][2] += Tr * olin[pp][ic];
                    acc[pp][ic][3] += Ti * olin[pp][ic];
                }
        }
#pragma unroll
        for (int pp = 0; pp < PC; ++pp) {
            const int p = p0 + pp;
            if (p >= O.n_probe) break;
#pragma unroll
            for (int ic = 0; ic < 6; ++ic) {
                if (ic < nc) {
                    const size_t k0 = ((((size_t)id * O.n_r + ir) * O.n_probe + p) * nc + ic) * 2;
                    avg_to[E.ato_off + ((k0 + 0) * S + s) * nsig + xs] =
                        make_double2(acc[pp][ic][0] * inv, acc[pp][ic][1] * inv);
                    avg_to[E.ato_off + ((k0 + 1) * S + s) * nsig + xs] =
                        make_double2(acc[pp][ic][2] * inv, acc[pp][ic][3] * inv);
                }
            }
        }
    }
}

hipError_t launch_contract(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, const ObsDesc* d_obs,
                           const int* d_r, const int* d_probe, const int* d_comp, const double2* hist_c,
                           const void* hist_o, double2* avg_t, double2* avg_to, int n_meas, int precision,
                           int max_slabs, int n_dirs, hipStream_t st)
{
    const dim3 g(total_blocks, max_slabs, n_dirs);
    if (precision == 0)
        hipLaunchKernelGGL(k_contract<double>, g, dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, d_r, d_probe, d_comp,
                           hist_c, (const double*)hist_o, avg_t, avg_to, n_meas);
    else
        hipLaunchKernelGGL(k_contract<float>, g, dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, d_r, d_probe, d_comp,
                           hist_c, (const float*)hist_o, avg_t, avg_to, n_meas);
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
// Slab products and sums over sites.  Block (e, r, probe): every thread walks
// (axis, x) in a fixed stride, forms P(x) = prod_S A(S) and
// W_S(x) = prod_{S' != S} A(S') as scaled complex numbers, and adds
// P (correlator, probe 0 only) and sum_S B(S) W_S (insertions) to
// double-double accumulators; a fixed-order tree reduces the block.
// src_t  = A * scale_t, src_to = B * scale_t (scale_t = 1 or 1/n_outer).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_product(const EnsDesc* __restrict__ ens, const ObsDesc* __restrict__ obs,
                                                 int n_pgroups, const double2* __restrict__ src_t,
                                                 const double2* __restrict__ src_to, int use_outer, double scale_t,
                                                 double* __restrict__ results, const int* __restrict__ ring)
{
    const int n_r = obs->n_r;
    const int e = blockIdx.x / (n_r * n_pgroups);
    const int ir = (blockIdx.x / n_pgroups) % n_r;
    const int p = blockIdx.x % n_pgroups;
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int nsig = E.nsig;
    const int S = use_outer ? E.s_out : E.s_in;
    const long long t_off = use_outer ? E.ot_off : E.at_off;
    const long long to_off = use_outer ? E.oto_off : E.ato_off;
    const int nc = O.n_comp;
    const bool has_probe = O.n_probe > 0;
    dd cre{0, 0}, cim{0, 0};
    dd ore[12], oim[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        ore[k] = dd{0, 0};
        oim[k] = dd{0, 0};
    }
    const int n_items = O.n_dirs * nsig;
    for (int it = threadIdx.x; it < n_items; it += blockDim.x) {
        const int id = it / nsig, xs = it - id * nsig;
        const size_t trow = ((size_t)id * n_r + ir) * S;
        sc P{1.0, 0.0, 0};
        for (int s = 0; s < S; ++s) {
            double2 a = src_t[t_off + (trow + s) * nsig + xs];
            a.x *= scale_t;
            a.y *= scale_t;
            P = sc_mul(P, a);
        }
        if (p == 0) {
            const double2 v = sc_val(P);
            cre = dd_add(cre, v.x);
            cim = dd_add(cim, v.y);
        }
        if (!has_probe) continue;
        for (int s = 0; s < S; ++s) {
            sc W{1.0, 0.0, 0};
            for (int s2 = 0; s2 < S; ++s2) {
                if (s2 == s) continue;
                double2 a = src_t[t_off + (trow + s2) * nsig + xs];
                a.x *= scale_t;
                a.y *= scale_t;
                W = sc_mul(W, a);
            }
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                if (k < 2 * nc) {
                    const size_t row = ((((size_t)id * n_r + ir) * O.n_probe + p) * nc) * 2 + k;
                    double2 b = src_to[to_off + (row * S + s) * nsig + xs];
                    b.x *= scale_t;
                    b.y *= scale_t;
                    const double2 v = sc_val(sc_mul(W, b));
                    ore[k] = dd_add(ore[k], v.x);
                    oim[k] = dd_add(oim[k], v.y);
                }
            }
        }
    }
    // fixed-order block reduction of each quantity
    __shared__ double shh[256], shl[256];
    const int slot = *ring;
    double* out = results + ((size_t)slot * gridDim.x / (n_r * n_pgroups) + e) * O.n_doubles_per_config;
    const double nC = 1.0 / ((double)nsig * O.n_dirs);
    const double nCO = nC / (double)E.nt;
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
    if (p == 0) {
        const dd a = reduce(cre), b = reduce(cim);
        if (threadIdx.x == 0) {
            out[2 * ir] = (a.hi + a.lo) * nC;
            out[2 * ir + 1] = (b.hi + b.lo) * nC;
        }
    }
    if (has_probe) {
        const long long base_co = 2ll * n_r;
        for (int k = 0; k < 2 * nc; ++k) {
            const dd a = reduce(ore[k]), b = reduce(oim[k]);
            if (threadIdx.x == 0) {
                const long long idx = (((long long)ir * O.n_probe + p) * nc) * 2 + k;
                out[base_co + 2 * idx] = (a.hi + a.lo) * nCO;
                out[base_co + 2 * idx + 1] = (b.hi + b.lo) * nCO;
            }
        }
    }
}

hipError_t launch_product(const EnsDesc* d_ens, int n_ens, const ObsDesc* d_obs, int n_r, int n_pgroups,
                          const double2* src_t, const double2* src_to, int use_outer, double scale, double* results,
                          const int* d_ring, hipStream_t st)
{
    hipLaunchKernelGGL(k_product, dim3(n_ens * n_r * n_pgroups), dim3(256), 0, st, d_ens, d_obs, n_pgroups, src_t,
                       src_to, use_outer, scale, results, d_ring);
    return hipGetLastError();
}

// vacuum <O_sq>, <O_lin> per orientation: the sum of every block partial of
// every measurement of the configuration (double-double, fixed order), divided
// by (measurements * V).  Block (e, k) reduces quantity k of ensemble e.
__global__ void __launch_bounds__(256) k_vac_final(const EnsDesc* __restrict__ ens, int n_ens,
                                                   const ObsDesc* __restrict__ obs, const double* __restrict__ vac_part,
                                                   int n_meas, double* __restrict__ results,
                                                   const int* __restrict__ ring)
{
    const int e = blockIdx.x / 12, k = blockIdx.x % 12;
    const EnsDesc& E = ens[e];
    const long long n = (long long)n_meas * E.n_vac_blocks;
    dd a{0.0, 0.0};
    for (long long i = threadIdx.x; i < n; i += blockDim.x) a = dd_add(a, vac_part[E.vac_part_off + i * 12 + k]);
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
        double* out = results + ((size_t)(*ring) * n_ens + e) * O.n_doubles_per_config;
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
