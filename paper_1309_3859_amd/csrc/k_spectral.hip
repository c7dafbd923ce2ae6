// k_spectral.hip -- the insertion estimators in spectral form.
//
// Paper: Amado, Cardoso, Bicudo, arXiv 1309.3859, Sec. II.C.3 (insertion
// estimator <P^dagger P O> = 1/(N_sigma N_t |M|) sum_x sum_mu sum_S [TO](S)
// prod_{S' != S} [T](S'), [TO] the slab average of T^(tau) times the slab
// sum of O at the probe site) and Sec. II.C.2 (two levels: T^(4), TO^(4)).
//
// Written out over the stored measurements m of every inner level k, with
// thin slab s inside thick slab S (one level: a single thick slab of all the
// slabs, and W = 1):
//   sum_x sum_S [TO](S) W_S = 1/(n_o n_i) sum_k sum_s sum_m sum_x G_k(x,s) T_m(x,s) O_m(x + d, s),
//   G_k(x, s) = W_S(x) prod_{s' in S, s' != s} [T]_k(x, s'),   W_S = prod_{S' != S} A(S'),
// A the outer averages.  For a charge axis, a slab, a separation and a
// component, the sum over x for every transverse displacement p = (p1, p2)
// at once is a cross-correlation over the plane orthogonal to the axis.  With
// the plane transform X^(k) = sum_{u,v} X(u,v) exp(-2 pi i (k1 u/n1 + k2 v/n2))
// and h^~ the transform with the conjugate kernel:
//   sum_x h(x) O(x + l e_par + p)
//     = 1/(n1 n2) sum_k exp(+2 pi i (k1 p1/n1 + k2 p2/n2)) sum_{x_par} O^_{x_par + l}(k) h^~_{x_par}(k).
// The inner sum is accumulated over measurements and inner levels per
// (axis, slab, r, component, kind, probe group); the probes' displacements
// are read off once per configuration.  Memory is independent of the number
// of probes.
#include "device_common.hpp"
#include "u1ml_internal.hpp"

namespace u1ml {

namespace {

__device__ inline int find_ens_s(const int* __restrict__ bstart, int n_ens, int bid)
{
    int e = 0;
    while (e + 1 < n_ens && bid >= bstart[e + 1]) ++e;
    return e;
}

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

__device__ inline int orient_of(int c, int dir) { return c < 3 ? (dir + c) % 3 : 3 + (dir + c - 3) % 3; }
__device__ inline bool spans_axis(int c) { return c == 0 || c == 4 || c == 5; }

struct dds {
    double hi, lo;
};

__device__ inline dds dds_add(dds a, double b)
{
    const double s = a.hi + b;
    const double bb = s - a.hi;
    const double err = (a.hi - (s - bb)) + (b - bb) + a.lo;
    const double hi = s + err;
    return dds{hi, err - (hi - s)};
}

}  // namespace

// ---------------------------------------------------------------------------
// Weights.  One work-item per (ensemble, axis, r, x); it writes every slab.
//   k_wfac: W[axis, r][S][x] = prod_{S' != S} scale * out_t[axis, r][S'][x]
//   k_gfac: G[axis, r][s][x] = W_S(x) prod_{s' in S, s' != s} avg_t[axis, r][s'][x]
//           (q thin slabs per thick slab, q = 0 for all slabs; W = 1 when wf is null)
// Products run over ascending slab index.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_wfac(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                              int n_ens, const ObsDesc* __restrict__ obs,
                                              const double2* __restrict__ out_t, double scale,
                                              double2* __restrict__ wf)
{
    const int e = find_ens_s(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const long long item = (long long)(blockIdx.x - bstart[e]) * blockDim.x + threadIdx.x;
    const int nsig = E.nsig, So = E.s_out;
    if (item >= (long long)obs->n_dirs * obs->n_r * nsig) return;
    const int xs = (int)(item % nsig);
    const long long idr = item / nsig;
    for (int S = 0; S < So; ++S) {
        double2 w = make_double2(1.0, 0.0);
        for (int S2 = 0; S2 < So; ++S2) {
            if (S2 == S) continue;
            double2 a = out_t[E.ot_off + ((size_t)idr * So + S2) * nsig + xs];
            a.x *= scale;
            a.y *= scale;
            w = cmul(w, a);
        }
        wf[E.wf_off + ((size_t)idr * So + S) * nsig + xs] = w;
    }
}

__global__ void __launch_bounds__(256) k_gfac(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                              int n_ens, const ObsDesc* __restrict__ obs,
                                              const double2* __restrict__ avg_t, const double2* __restrict__ wf,
                                              int q, double2* __restrict__ gf)
{
    const int e = find_ens_s(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const long long item = (long long)(blockIdx.x - bstart[e]) * blockDim.x + threadIdx.x;
    const int nsig = E.nsig, Si = E.s_in, So = E.s_out;
    if (item >= (long long)obs->n_dirs * obs->n_r * nsig) return;
    const int xs = (int)(item % nsig);
    const long long idr = item / nsig;
    const int qq = q > 0 ? q : Si;  // q = 0: one thick slab of every slab (one level)
    for (int s = 0; s < Si; ++s) {
        const int S = s / qq;
        double2 g = wf ? wf[E.wf_off + ((size_t)idr * So + S) * nsig + xs] : make_double2(1.0, 0.0);
        for (int s2 = S * qq; s2 < S * qq + qq; ++s2) {
            if (s2 == s) continue;
            g = cmul(g, avg_t[E.at_off + ((size_t)idr * Si + s2) * nsig + xs]);
        }
        gf[E.gf_off + ((size_t)idr * Si + s) * nsig + xs] = g;
    }
}

// One axis of the plane transform, in LDS:
//   out[a oa + b ob] = sum_c in[a sa + c sc] tw[(b c) mod nc],  a < na, b < nc,
// every thread owning a TxT tile of (a, b) so that each loaded input and
// twiddle serves T products.  na and nc are multiples of T.
template <int T>
__device__ inline void dft_axis(const double2* __restrict__ in, int na, int nc, int sa, int sc,
                                const double2* __restrict__ tw, double2* __restrict__ out, int oa, int ob)
{
    const int nbt = nc / T;
    const int tiles = (na / T) * nbt;
    for (int t = threadIdx.x; t < tiles; t += blockDim.x) {
        const int a0 = (t / nbt) * T, b0 = (t - (t / nbt) * nbt) * T;
        double re[T][T], im[T][T];
        int ph[T];
#pragma unroll
        for (int j = 0; j < T; ++j) {
            ph[j] = 0;
#pragma unroll
            for (int i = 0; i < T; ++i) re[i][j] = im[i][j] = 0.0;
        }
        for (int c = 0; c < nc; ++c) {
            double2 x[T], w[T];
#pragma unroll
            for (int i = 0; i < T; ++i) x[i] = in[(a0 + i) * sa + c * sc];
#pragma unroll
            for (int j = 0; j < T; ++j) {
                w[j] = tw[ph[j]];
                ph[j] += b0 + j;
                if (ph[j] >= nc) ph[j] -= nc;
            }
#pragma unroll
            for (int i = 0; i < T; ++i)
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    re[i][j] += x[i].x * w[j].x - x[i].y * w[j].y;
                    im[i][j] += x[i].x * w[j].y + x[i].y * w[j].x;
                }
        }
#pragma unroll
        for (int i = 0; i < T; ++i)
#pragma unroll
            for (int j = 0; j < T; ++j) out[(a0 + i) * oa + (b0 + j) * ob] = make_double2(re[i][j], im[i][j]);
    }
}

// ---------------------------------------------------------------------------
// Plane transforms of measurement m_in.  Work-group per (ensemble, axis,
// slab s, field f, axis coordinate x_par); fields f < n_r are
// h = G(x,s,r) conj(c_m(x)) c_m(x + r e_par) (conjugate kernel), fields
// n_r .. n_r + 11 the O rows (orientation, kind) (plain kernel).  The plane
// is staged in LDS, transformed along v, then along u; twiddles
// exp(2 pi i j / n) come from sincospi in FP64.  Each output is a sum over
// the axis in ascending order, whatever the tile shape.
//   sph[axis][s][r][x_par][k],  spo[axis][s][row][x_par][k],  k = k1 n2 + k2
// ---------------------------------------------------------------------------
template <typename ot, int T>
__global__ void __launch_bounds__(256) k_dft_planes(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                    int n_ens, const ObsDesc* __restrict__ obs,
                                                    const int* __restrict__ rlist, const double2* __restrict__ hist_c,
                                                    const ot* __restrict__ hist_o, const double2* __restrict__ gf,
                                                    double2* __restrict__ sph, double2* __restrict__ spo, int m_in)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int e = find_ens_s(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int nsig = E.nsig, Si = E.s_in, R = O.n_r, NF = R + 12;
    const int n3[3] = {E.nx, E.ny, E.nz};
    const int npm = max(E.nx, max(E.ny, E.nz));
    int local = blockIdx.x - bstart[e];
    const int xpar = local % npm;
    local /= npm;
    const int f = local % NF;
    local /= NF;
    const int s = local % Si;
    const int id = local / Si;
    if (id >= O.n_dirs) return;
    const int dir = O.dirs[id];
    const int N = n3[dir];
    if (xpar >= N) return;  // uniform for the block
    const int d1 = dir == 2 ? 0 : dir + 1, d2 = dir == 0 ? 2 : dir - 1;
    const int n1 = n3[d1], n2 = n3[d2], n12 = n1 * n2;
    double2* X = reinterpret_cast<double2*>(lds_raw);
    double2* Y = X + n12;
    double2* w1 = Y + n12;
    double2* w2 = w1 + n1;
    const double sg = f < R ? 1.0 : -1.0;  // sign of the kernel's exponent
    for (int j = threadIdx.x; j < n1; j += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)j / (double)n1, &sn, &cs);
        w1[j] = make_double2(cs, sg * sn);
    }
    for (int j = threadIdx.x; j < n2; j += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)j / (double)n2, &sn, &cs);
        w2[j] = make_double2(cs, sg * sn);
    }
    // stride of each lattice axis in the site index x + nx (y + ny z)
    const int st3[3] = {1, E.nx, E.nx * E.ny};
    const int base = xpar * st3[dir];
    if (f < R) {
        const int r = rlist[f];
        const int xr_off = ((xpar + r) % N - xpar) * st3[dir];
        const double2* hc = hist_c + E.hc_off + ((size_t)m_in * Si + s) * nsig;
        const double2* g = gf + E.gf_off + (((size_t)id * R + f) * Si + s) * nsig;
        for (int j = threadIdx.x; j < n12; j += blockDim.x) {
            const int u = j / n2, v = j - u * n2;
            const int xs = base + u * st3[d1] + v * st3[d2];
            const double2 a = hc[xs], b = hc[xs + xr_off];
            const double2 t = make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
            X[j] = cmul(g[xs], t);
        }
    } else {
        const ot* ho = hist_o + E.ho_off + (((size_t)m_in * Si + s) * 12 + (f - R)) * nsig;
        for (int j = threadIdx.x; j < n12; j += blockDim.x) {
            const int u = j / n2, v = j - u * n2;
            X[j] = make_double2((double)ho[base + u * st3[d1] + v * st3[d2]], 0.0);
        }
    }
    __syncthreads();
    // along v, then along u (tiles of T x T outputs per thread)
    dft_axis<T>(X, n1, n2, n2, 1, w2, Y, n2, 1);
    __syncthreads();
    double2* out = f < R ? sph + E.sph_off + (((size_t)id * Si + s) * R + f) * nsig + (size_t)xpar * n12
                         : spo + E.spo_off + (((size_t)id * Si + s) * 12 + (f - R)) * nsig + (size_t)xpar * n12;
    dft_axis<T>(Y, n2, n1, 1, n2, w1, out, 1, n2);
}

// ---------------------------------------------------------------------------
// Spectral sums of one measurement.  One work-item per (ensemble, axis, slab,
// r, component, kind, probe group, k):
//   F[...][k] += sum_{x_par} O^_{row}(x_par + l) (k) * h^~_r(x_par) (k)
// with l = l_g + (mode_g ? l_mid(r, c) : 0) and row = 2 o(c, axis) + kind.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_spec_mac(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                  int n_ens, const ObsDesc* __restrict__ obs,
                                                  const int* __restrict__ rlist, const int* __restrict__ comps,
                                                  const int* __restrict__ gdesc, const double2* __restrict__ sph,
                                                  const double2* __restrict__ spo, double2* __restrict__ facc)
{
    const int e = find_ens_s(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int nsig = E.nsig, Si = E.s_in, R = O.n_r, Nc = O.n_comp, NG = O.n_groups;
    const int n3[3] = {E.nx, E.ny, E.nz};
    int n12max = 0;
    for (int i = 0; i < O.n_dirs; ++i) n12max = max(n12max, nsig / n3[O.dirs[i]]);
    long long item = (long long)(blockIdx.x - bstart[e]) * blockDim.x + threadIdx.x;
    const long long total = (long long)O.n_dirs * Si * R * Nc * 2 * NG * n12max;
    if (item >= total) return;
    const long long slot = item / n12max;  // ((((id Si + s) R + ir) Nc + ic) 2 + kind) NG + g
    const int k = (int)(item - slot * n12max);
    long long t = slot;
    const int g = (int)(t % NG);
    t /= NG;
    const int kind = (int)(t % 2);
    t /= 2;
    const int ic = (int)(t % Nc);
    t /= Nc;
    const int ir = (int)(t % R);
    t /= R;
    const int s = (int)(t % Si);
    const int id = (int)(t / Si);
    const int dir = O.dirs[id];
    const int N = n3[dir], n12 = nsig / N;
    if (k >= n12) return;
    const int c = comps[ic], r = rlist[ir];
    const int l = gdesc[2 * g] + (gdesc[2 * g + 1] ? (spans_axis(c) ? (r - 1) / 2 : r / 2) : 0);
    const int row = 2 * orient_of(c, dir) + kind;
    const double2* h = sph + E.sph_off + (((size_t)id * Si + s) * R + ir) * nsig + k;
    const double2* o = spo + E.spo_off + (((size_t)id * Si + s) * 12 + row) * nsig + k;
    int xo = ((l % N) + N) % N;
    double re = 0.0, im = 0.0;
    for (int xp = 0; xp < N; ++xp) {
        const double2 a = o[(size_t)xo * n12], b = h[(size_t)xp * n12];
        re += a.x * b.x - a.y * b.y;
        im += a.x * b.y + a.y * b.x;
        if (++xo == N) xo = 0;
    }
    double2* F = facc + E.facc_off + (size_t)slot * n12max + k;
    *F = make_double2(F->x + re, F->y + im);
}

// ---------------------------------------------------------------------------
// Probe estimates of the configuration.  One work-item per (ensemble, r,
// probe, component, kind):
//   CO = scale sum_axis 1/(n1 n2) sum_s sum_k F[axis][s][r][c][kind][g(p)][k] exp(+2 pi i (k1 p1/n1 + k2 p2/n2))
// in double-double, k ascending; scale = 1/(N_sigma |M| N_t n_o n_i).  The
// twiddle tables exp(2 pi i j / n) of each axis are shared in LDS by the
// work-group (dynamic LDS: 2 max(Nx, Ny, Nz) double2).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_spec_final(const EnsDesc* __restrict__ ens, int n_ens,
                                                   const ObsDesc* __restrict__ obs, const int* __restrict__ probes,
                                                   const int* __restrict__ pgroup, const double2* __restrict__ facc,
                                                   double n_meas_total, double* __restrict__ results,
                                                   const int* __restrict__ ring)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ObsDesc& O = *obs;
    const int R = O.n_r, Np = O.n_probe, Nc = O.n_comp, NG = O.n_groups;
    const long long per = (long long)R * Np * Nc * 2;
    const int blocks_per_ens = (int)((per + blockDim.x - 1) / blockDim.x);
    const int e = blockIdx.x / blocks_per_ens;  // uniform for the block
    if (e >= n_ens) return;
    const long long t0 = (long long)(blockIdx.x - e * blocks_per_ens) * blockDim.x + threadIdx.x;
    const bool valid = t0 < per;
    long long t = valid ? t0 : 0;  // ((ir Np + p) Nc + ic) 2 + kind
    const int kind = (int)(t % 2);
    t /= 2;
    const int ic = (int)(t % Nc);
    t /= Nc;
    const int p = (int)(t % Np);
    const int ir = (int)(t / Np);
    const EnsDesc& E = ens[e];
    const int nsig = E.nsig, Si = E.s_in;
    const int n3[3] = {E.nx, E.ny, E.nz};
    const int npm = max(E.nx, max(E.ny, E.nz));
    double2* w1 = reinterpret_cast<double2*>(lds_raw);
    double2* w2 = w1 + npm;
    int n12max = 0;
    for (int k = 0; k < O.n_dirs; ++k) n12max = max(n12max, nsig / n3[O.dirs[k]]);
    const int g = pgroup[p], p1 = probes[4 * p + 1], p2 = probes[4 * p + 2];
    dds are{0.0, 0.0}, aim{0.0, 0.0};
    for (int id = 0; id < O.n_dirs; ++id) {
        const int dir = O.dirs[id];
        const int d1 = dir == 2 ? 0 : dir + 1, d2 = dir == 0 ? 2 : dir - 1;
        const int n1 = n3[d1], n2 = n3[d2], n12 = n1 * n2;
        __syncthreads();
        for (int j = threadIdx.x; j < n1; j += blockDim.x) {
            double sn, cs;
            sincospi(2.0 * (double)j / (double)n1, &sn, &cs);
            w1[j] = make_double2(cs, sn);
        }
        for (int j = threadIdx.x; j < n2; j += blockDim.x) {
            double sn, cs;
            sincospi(2.0 * (double)j / (double)n2, &sn, &cs);
            w2[j] = make_double2(cs, sn);
        }
        __syncthreads();
        if (!valid) continue;
        const double inv = 1.0 / (double)n12;
        const int q1 = ((p1 % n1) + n1) % n1, q2 = ((p2 % n2) + n2) % n2;
        for (int s = 0; s < Si; ++s) {
            const size_t slot = (((((size_t)id * Si + s) * R + ir) * Nc + ic) * 2 + kind) * NG + g;
            const double2* F = facc + E.facc_off + slot * n12max;
            int ph1 = 0;
            for (int k1 = 0; k1 < n1; ++k1) {
                const double2 a = w1[ph1];
                int ph2 = 0;
                for (int k2 = 0; k2 < n2; ++k2) {
                    const double2 w = cmul(a, w2[ph2]);
                    const double2 v = F[k1 * n2 + k2];
                    are = dds_add(are, (v.x * w.x - v.y * w.y) * inv);
                    aim = dds_add(aim, (v.x * w.y + v.y * w.x) * inv);
                    ph2 += q2;
                    if (ph2 >= n2) ph2 -= n2;
                }
                ph1 += q1;
                if (ph1 >= n1) ph1 -= n1;
            }
        }
    }
    if (!valid) return;
    const double scale = 1.0 / ((double)nsig * O.n_dirs * E.nt * n_meas_total);
    double* out = results + ((size_t)(*ring) * O.n_ens_total + E.res_index) * O.n_doubles_per_config;
    const long long idx = (((long long)ir * Np + p) * Nc + ic) * 2 + kind;
    out[2ll * R + 2 * idx] = (are.hi + are.lo) * scale;
    out[2ll * R + 2 * idx + 1] = (aim.hi + aim.lo) * scale;
}

// element copy in 16-byte units (the replay's copy of the links; a kernel so
// that captured graphs hold no memset or memcpy nodes)
__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_wfac(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, const ObsDesc* d_obs,
                       const double2* out_t, double scale, double2* wf, hipStream_t st)
{
    hipLaunchKernelGGL(k_wfac, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, out_t, scale, wf);
    return hipGetLastError();
}

hipError_t launch_gfac(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, const ObsDesc* d_obs,
                       const double2* avg_t, const double2* wf, int q, double2* gf, hipStream_t st)
{
    hipLaunchKernelGGL(k_gfac, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, avg_t, wf, q, gf);
    return hipGetLastError();
}

// tile: 4 when every transverse extent is a multiple of 4, else 2 (extents are even)
hipError_t launch_dft_planes(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, size_t lds_bytes,
                             const ObsDesc* d_obs, const int* d_r, const double2* hist_c, const void* hist_o,
                             const double2* gf, double2* sph, double2* spo, int m_in, int precision, int tile,
                             hipStream_t st)
{
    const dim3 g(total_blocks), b(256);
    if (precision == 0) {
        if (tile == 4)
            hipLaunchKernelGGL((k_dft_planes<double, 4>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               hist_c, (const double*)hist_o, gf, sph, spo, m_in);
        else
            hipLaunchKernelGGL((k_dft_planes<double, 2>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               hist_c, (const double*)hist_o, gf, sph, spo, m_in);
    } else {
        if (tile == 4)
            hipLaunchKernelGGL((k_dft_planes<float, 4>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               hist_c, (const float*)hist_o, gf, sph, spo, m_in);
        else
            hipLaunchKernelGGL((k_dft_planes<float, 2>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               hist_c, (const float*)hist_o, gf, sph, spo, m_in);
    }
    return hipGetLastError();
}

hipError_t launch_spec_mac(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks,
                           const ObsDesc* d_obs, const int* d_r, const int* d_comp, const int* d_gdesc,
                           const double2* sph, const double2* spo, double2* facc, hipStream_t st)
{
    hipLaunchKernelGGL(k_spec_mac, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, d_r, d_comp,
                       d_gdesc, sph, spo, facc);
    return hipGetLastError();
}

// n_outputs: outputs per ensemble (n_r n_probe n_comp 2); npm: largest lattice extent
hipError_t launch_spec_final(const EnsDesc* d_ens, int n_ens, const ObsDesc* d_obs, long long n_outputs, int npm,
                             const int* d_probe, const int* d_pgroup, const double2* facc, double n_meas_total,
                             double* results, const int* d_ring, hipStream_t st)
{
    if (n_outputs <= 0) return hipSuccess;
    const unsigned per_ens = (unsigned)((n_outputs + 63) / 64);
    hipLaunchKernelGGL(k_spec_final, dim3(per_ens * (unsigned)n_ens), dim3(64), 2 * (size_t)npm * sizeof(double2), st,
                       d_ens, n_ens, d_obs, d_probe, d_pgroup, facc, n_meas_total, results, d_ring);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    size_t g = (n16 + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)g), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

}  // namespace u1ml
