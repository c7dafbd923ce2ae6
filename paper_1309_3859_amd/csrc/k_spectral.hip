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
#include "scaled.hpp"
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

// Position of site xs = x + nx (y + ny z) in the plane-major order of charge
// axis dir: (x_par n1 + u) n2 + v, with (x_par, u, v) the coordinates along
// (dir, d1, d2), d1 = dir + 1 and d2 = dir + 2 (mod 3); each plane x_par is
// then one contiguous run of n1 n2 sites.
__device__ inline int plane_index(int xs, int dir, int nx, int ny, int nz)
{
    const int x = xs % nx, yz = xs / nx;
    const int y = yz % ny, z = yz / ny;
    const int xp = dir == 0 ? x : dir == 1 ? y : z;
    const int u = dir == 0 ? y : dir == 1 ? z : x;
    const int v = dir == 0 ? z : dir == 1 ? x : y;
    const int n1 = dir == 0 ? ny : dir == 1 ? nz : nx;
    const int n2 = dir == 0 ? nz : dir == 1 ? nx : ny;
    return (xp * n1 + u) * n2 + v;
}

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
//   k_wfac: W[axis, r][S][x] = 2^-E(r) prod_{S' != S} scale * out_t[axis, r][S'][x]
//   k_gfac: G[axis, r][s][x] = W_S(x) prod_{s' in S, s' != s} avg_t[axis, r][s'][x]
//           (q thin slabs per thick slab, q = 0 for all slabs; W = 2^-E(r) when
//           wf is null), stored in the plane-major order of the axis (plane_index)
// E(r) is the exponent of the configuration's correlator products, read from
// its record, so that the spectral sums come out relative to the same 2^E(r)
// as the correlator.  The products over slabs run as scaled complex numbers,
// over ascending slab index.
// ---------------------------------------------------------------------------
__device__ inline int record_exp(const EnsDesc& E, const ObsDesc& O, const double* __restrict__ results,
                                 const int* __restrict__ ring, int ir)
{
    const double* rec = results + ((size_t)(*ring) * O.n_ens_total + E.res_index) * O.n_doubles_per_config;
    return (int)rec[O.n_doubles_per_config - O.n_r + ir];
}

__global__ void __launch_bounds__(256) k_wfac(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                              int n_ens, const ObsDesc* __restrict__ obs,
                                              const double2* __restrict__ out_t, double scale,
                                              double2* __restrict__ wf, const double* __restrict__ results,
                                              const int* __restrict__ ring)
{
    const int e = find_ens_s(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const long long item = (long long)(blockIdx.x - bstart[e]) * blockDim.x + threadIdx.x;
    const int nsig = E.nsig, So = E.s_out;
    if (item >= (long long)obs->n_dirs * obs->n_r * nsig) return;
    const int xs = (int)(item % nsig);
    const long long idr = item / nsig;
    const int Er = record_exp(E, *obs, results, ring, (int)(idr % obs->n_r));
    for (int S = 0; S < So; ++S) {
        sc w{1.0, 0.0, 0};
        for (int S2 = 0; S2 < So; ++S2) {
            if (S2 == S) continue;
            double2 a = out_t[E.ot_off + ((size_t)idr * So + S2) * nsig + xs];
            a.x *= scale;
            a.y *= scale;
            w = sc_mul(w, a);
        }
        wf[E.wf_off + ((size_t)idr * So + S) * nsig + xs] = sc_rel(w, Er);
    }
}

__global__ void __launch_bounds__(256) k_gfac(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                              int n_ens, const ObsDesc* __restrict__ obs,
                                              const double2* __restrict__ avg_t, const double2* __restrict__ wf,
                                              int q, double2* __restrict__ gf, const double* __restrict__ results,
                                              const int* __restrict__ ring)
{
    const int e = find_ens_s(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const long long item = (long long)(blockIdx.x - bstart[e]) * blockDim.x + threadIdx.x;
    const int nsig = E.nsig, Si = E.s_in, So = E.s_out;
    if (item >= (long long)obs->n_dirs * obs->n_r * nsig) return;
    const int xs = (int)(item % nsig);
    const long long idr = item / nsig;
    const int qq = q > 0 ? q : Si;  // q = 0: one thick slab of every slab (one level)
    const int pidx = plane_index(xs, obs->dirs[idr / obs->n_r], E.nx, E.ny, E.nz);
    const int Er = wf ? 0 : record_exp(E, *obs, results, ring, (int)(idr % obs->n_r));
    for (int s = 0; s < Si; ++s) {
        const int S = s / qq;
        sc g{1.0, 0.0, 0};
        if (wf) {
            const double2 w = wf[E.wf_off + ((size_t)idr * So + S) * nsig + xs];
            g = sc{w.x, w.y, 0};
        }
        for (int s2 = S * qq; s2 < S * qq + qq; ++s2) {
            if (s2 == s) continue;
            g = sc_mul(g, avg_t[E.at_off + ((size_t)idr * Si + s2) * nsig + xs]);
        }
        gf[E.gf_off + ((size_t)idr * Si + s) * nsig + pidx] = sc_rel(g, Er);
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
// Mixed-radix FFT along one axis of a plane in LDS (Stockham autosort, radices
// 4, 2, 3, 5 in that order; Cooley & Tukey 1965, Stockham 1966).  Stage with
// radix R after the radices so far have product Ns: butterfly j of a sequence
// of length n takes the R inputs j + r n/R, multiplies input r by
// w^(r (j mod Ns) n/(Ns R)), forms their length-R transform and writes output
// q to (j div Ns) Ns R + (j mod Ns) + q Ns; after the last stage the sequence
// holds its transform in natural order.  w = exp(sg 2 pi i / n) comes from the
// table tw (n entries), so the forward and the conjugate kernel share the
// code.  Results differ from the direct sum only by rounding, and are the same
// for every launch shape.
// ---------------------------------------------------------------------------
struct FftPlan {
    int c4, c2, c3, c5;  // stages of each radix, applied in this order
    int n_st;            // total, 0 if n has a prime factor above 5
};

__device__ inline FftPlan fft_plan(int n)
{
    FftPlan p{0, 0, 0, 0, 0};
    while (n % 4 == 0) { ++p.c4; n /= 4; }
    while (n % 2 == 0) { ++p.c2; n /= 2; }
    while (n % 3 == 0) { ++p.c3; n /= 3; }
    while (n % 5 == 0) { ++p.c5; n /= 5; }
    p.n_st = n == 1 ? p.c4 + p.c2 + p.c3 + p.c5 : 0;
    return p;
}

// One stage over `rows` sequences: element i of sequence q at src[q sq + i se],
// written to dst[q dq + i de].  Consecutive work-items take consecutive
// butterflies of one sequence when the elements of a sequence are adjacent
// (se = 1), else the same butterfly of consecutive sequences (sq = 1), so the
// 16-byte LDS accesses of a wave stay on distinct banks and the last stage's
// global stores are contiguous.
// NC, RC, SC: the length, the number of sequences and Ns as compile-time
// constants (0: taken from the arguments), so that a fixed plane size folds
// the index arithmetic
template <int R, int NC = 0, int RC = 0, int SC = 0>
__device__ inline void fft_stage(const double2* __restrict__ src, int sq, int se, double2* __restrict__ dst, int dq,
                                 int de, int n_, int rows_, int Ns_, const double2* __restrict__ tw, double sg)
{
    const int n = NC ? NC : n_, rows = RC ? RC : rows_, Ns = SC ? SC : Ns_;
    const int m = n / R;
    const int tstep = n / (Ns * R);
    const int total = rows * m;
    const bool qfast = se != 1;
    for (int b = threadIdx.x; b < total; b += blockDim.x) {
        const int q = qfast ? b % rows : b / m;
        const int j = qfast ? b / rows : b - q * m;
        const int k = j % Ns;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[q * sq + (j + r * m) * se];
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * tstep]);  // r k tstep < n
        double2 V[R];
        if (R == 2) {
            V[0] = make_double2(v[0].x + v[1].x, v[0].y + v[1].y);
            V[1] = make_double2(v[0].x - v[1].x, v[0].y - v[1].y);
        } else if (R == 4) {
            // w_4 = sg i: w z = sg (-z.y, z.x)
            const double2 a = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
            const double2 c = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
            const double2 bb = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
            const double2 d = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
            const double2 wd = make_double2(-sg * d.y, sg * d.x);
            V[0] = make_double2(a.x + bb.x, a.y + bb.y);
            V[1] = make_double2(c.x + wd.x, c.y + wd.y);
            V[2] = make_double2(a.x - bb.x, a.y - bb.y);
            V[3] = make_double2(c.x - wd.x, c.y - wd.y);
        } else {
            const int nr = n / R;
#pragma unroll
            for (int qq = 0; qq < R; ++qq) {
                double2 acc = v[0];
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const double2 w = tw[((r * qq) % R) * nr];
                    acc.x += v[r].x * w.x - v[r].y * w.y;
                    acc.y += v[r].x * w.y + v[r].y * w.x;
                }
                V[qq] = acc;
            }
        }
        const int idx = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int qq = 0; qq < R; ++qq) dst[q * dq + (idx + qq * Ns) * de] = V[qq];
    }
}

// The whole FFT along one axis: input in LDS buffer `cur` (sequence stride sq,
// element stride se), stages ping-pong between `cur` and `other` (same
// strides), the last stage writes to out[q oq + k oe] (global memory, or the
// LDS buffer that the last stage does not read).
__device__ inline void fft_axis(const FftPlan& P, double2* cur, double2* other, int sq, int se, int n, int rows,
                                const double2* tw, double sg, double2* out, int oq, int oe)
{
    int Ns = 1;
    for (int st = 0; st < P.n_st; ++st) {
        const bool last = st == P.n_st - 1;
        double2* dst = last ? out : other;
        const int dq = last ? oq : sq, de = last ? oe : se;
        const int R = st < P.c4 ? 4 : st < P.c4 + P.c2 ? 2 : st < P.c4 + P.c2 + P.c3 ? 3 : 5;
        switch (R) {
        case 4: fft_stage<4>(cur, sq, se, dst, dq, de, n, rows, Ns, tw, sg); break;
        case 2: fft_stage<2>(cur, sq, se, dst, dq, de, n, rows, Ns, tw, sg); break;
        case 3: fft_stage<3>(cur, sq, se, dst, dq, de, n, rows, Ns, tw, sg); break;
        default: fft_stage<5>(cur, sq, se, dst, dq, de, n, rows, Ns, tw, sg); break;
        }
        __syncthreads();
        Ns *= R;
        double2* t = cur;
        cur = other;
        other = t;
    }
}

// The same FFT for an axis of compile-time length N on an N x N plane: the
// stages of fft_plan(N) in the same order with the same arithmetic, every
// length, count and stride constant.
__host__ __device__ constexpr int cplan_stage(int n, int st, bool want_ns)
{
    int i = 0, ns = 1;
    const int radices[4] = {4, 2, 3, 5};
    for (int ri = 0; ri < 4; ++ri) {
        const int r = radices[ri];
        while (n % r == 0) {
            if (i == st) return want_ns ? ns : r;
            ++i;
            ns *= r;
            n /= r;
        }
    }
    return want_ns ? ns : (n == 1 ? -i : 0);  // past the last stage: minus the stage count
}
__host__ __device__ constexpr int cplan_nst(int n) { return -cplan_stage(n, 64, false); }

template <int N, int ST>
__device__ inline void fft_axis_c(double2* cur, double2* other, int sq, int se, const double2* tw, double sg,
                                  double2* out, int oq, int oe)
{
    constexpr int NST = cplan_nst(N);
    if constexpr (ST < NST) {
        constexpr int R = cplan_stage(N, ST, false), NS = cplan_stage(N, ST, true);
        constexpr bool last = ST == NST - 1;
        fft_stage<R, N, N, NS>(cur, sq, se, last ? out : other, last ? oq : sq, last ? oe : se, N, N, NS, tw, sg);
        __syncthreads();
        fft_axis_c<N, ST + 1>(other, cur, sq, se, tw, sg, out, oq, oe);
    }
}

// ---------------------------------------------------------------------------
// Staging of measurement m_in for the plane transforms: the slab phases and
// the 12 O rows copied to the plane-major order of each charge axis, so that
// every plane the transforms read is contiguous.
//   cpl[axis][s][plane_index],  opl[axis][s][row][plane_index]
// Work-group per (ensemble, axis, slab, tile): the target's fastest
// coordinate is v (z for the x axis, x for the y axis, y for the z axis); a
// tile is 32 x values by 32 v values at fixed remaining coordinate, read with
// x fastest and written with v fastest through LDS (the slab phase and four O
// rows per pass), so both sides are contiguous.  For the y axis (v = x) the
// tile is 32 x values of 32 rows, copied directly.
// ---------------------------------------------------------------------------
constexpr int kStageTile = 32;

template <typename ot>
__global__ void __launch_bounds__(256) k_plane_stage(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                     int n_ens, const ObsDesc* __restrict__ obs,
                                                     const double2* __restrict__ hist_c, const ot* __restrict__ hist_o,
                                                     int m_in, double2* __restrict__ cpl, ot* __restrict__ opl)
{
    constexpr int TT = kStageTile;
    __shared__ double2 tc[TT][TT + 1];
    __shared__ ot to[4][TT][TT + 1];  // four O rows per pass
    const int e = find_ens_s(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int nx = E.nx, ny = E.ny, nz = E.nz, nsig = E.nsig, Si = E.s_in;
    const int npm = max(nx, max(ny, nz));
    const int tx_n = (nx + TT - 1) / TT, tv_n = (npm + TT - 1) / TT;
    const int tiles = tx_n * tv_n * npm;  // per (axis, slab), sized for the largest extent
    int local = blockIdx.x - bstart[e];
    const int tile = local % tiles;
    local /= tiles;
    const int s = local % Si;
    const int id = local / Si;
    if (id >= O.n_dirs) return;
    const int dir = O.dirs[id];
    // v: the target's fastest axis; w: the remaining one (y axis: v = x, rows y, w = z)
    const int vax = dir == 0 ? 2 : dir == 1 ? 0 : 1;
    const int wax = dir == 0 ? 1 : 2;
    const int n3[3] = {nx, ny, nz};
    const int nrow = vax == 0 ? ny : n3[vax];  // extent of the tile's second index
    const int x0 = (tile % tx_n) * TT;
    const int v0 = ((tile / tx_n) % tv_n) * TT;
    const int w = tile / (tx_n * tv_n);
    if (w >= n3[wax] || v0 >= nrow) return;  // uniform for the block
    const size_t ps = (size_t)id * Si + s;
    const double2* hc = hist_c + E.hc_off + ((size_t)m_in * Si + s) * nsig;
    const ot* ho = hist_o + E.ho_off + ((size_t)m_in * Si + s) * 12 * nsig;
    double2* dc = cpl + E.cpl_off + ps * nsig;
    ot* dob = opl + E.opl_off + ps * 12 * nsig;
    const int lx = threadIdx.x % TT, ly = threadIdx.x / TT;  // 32 x 8 work-items
    if (vax == 0) {
        // y axis: plane index (y nz + z) nx + x keeps x fastest: a plain copy of 32 rows
        for (int i = ly; i < TT; i += 8) {
            const int y = v0 + i, x = x0 + lx;
            if (y >= ny || x >= nx) continue;
            const int xs = x + nx * (y + ny * w);
            const int p = (y * nz + w) * nx + x;
            dc[p] = hc[xs];
#pragma unroll
            for (int row = 0; row < 12; ++row) dob[(size_t)row * nsig + p] = ho[(size_t)row * nsig + xs];
        }
        return;
    }
    for (int pass = 0; pass < 3; ++pass) {
        // read with x fastest
        for (int i = ly; i < TT; i += 8) {
            const int v = v0 + i, x = x0 + lx;
            if (v < nrow && x < nx) {
                const int y = vax == 1 ? v : w, z = vax == 2 ? v : w;
                const int xs = x + nx * (y + ny * z);
                if (pass == 0) tc[i][lx] = hc[xs];
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) to[r4][i][lx] = ho[(size_t)(4 * pass + r4) * nsig + xs];
            }
        }
        __syncthreads();
        // write with v fastest: x axis p = (x ny + y) nz + z (y = w, z = v); z axis p = (z nx + x) ny + y (z = w, y = v)
        for (int i = ly; i < TT; i += 8) {
            const int x = x0 + i, v = v0 + lx;
            if (v < nrow && x < nx) {
                const int p = vax == 2 ? (x * ny + w) * nz + v : (w * nx + x) * ny + v;
                if (pass == 0) dc[p] = tc[lx][i];
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) dob[(size_t)(4 * pass + r4) * nsig + p] = to[r4][lx][i];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Plane transforms of measurement m_in.  Work-group per (ensemble, axis,
// slab s, field f, axis coordinate x_par); fields f < n_r are
// h = G(x,s,r) conj(c_m(x)) c_m(x + r e_par) (conjugate kernel), fields
// n_r .. n_r + 11 the O rows (orientation, kind) (plain kernel).  The plane
// is staged in LDS, transformed along v, then along u, by the mixed-radix
// FFT when both extents factor into 2, 3 and 5, else by direct sums over the
// axis in ascending order; twiddles exp(2 pi i j / n) come from sincospi in
// FP64.  Either way the outputs are the same for every launch shape.
//   sph[axis][s][r][x_par][k],  spo[axis][s][row][x_par][k],  k = k1 n2 + k2
// ---------------------------------------------------------------------------
constexpr int kPlaneThreads = 512;  // two work-groups fill a CU's LDS; more threads per plane hide latency

template <typename ot, int T, int NP>
__global__ void __launch_bounds__(kPlaneThreads) k_dft_planes(const EnsDesc* __restrict__ ens, const int* __restrict__ bstart,
                                                    int n_ens, const ObsDesc* __restrict__ obs,
                                                    const int* __restrict__ rlist, const double2* __restrict__ cpl,
                                                    const ot* __restrict__ opl, const double2* __restrict__ gf,
                                                    double2* __restrict__ sph, double2* __restrict__ spo)
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
    // the staged measurement and G are in plane-major order: plane x_par is
    // the contiguous run [x_par n12, (x_par + 1) n12)
    const size_t ps = (size_t)id * Si + s;
    if (f < R) {
        const int r = rlist[f];
        const double2* ca = cpl + E.cpl_off + ps * nsig + (size_t)xpar * n12;
        const double2* cb = cpl + E.cpl_off + ps * nsig + (size_t)((xpar + r) % N) * n12;
        const double2* g = gf + E.gf_off + (((size_t)id * R + f) * Si + s) * nsig + (size_t)xpar * n12;
        // four elements per work-item and round, all loads issued before any use
        for (int j0 = threadIdx.x; j0 < n12; j0 += 4 * blockDim.x) {
            double2 a[4], b[4], gg[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = min(j0 + u * (int)blockDim.x, n12 - 1);
                a[u] = ca[j];
                b[u] = cb[j];
                gg[u] = g[j];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u * (int)blockDim.x;
                const double2 t = make_double2(a[u].x * b[u].x + a[u].y * b[u].y, a[u].x * b[u].y - a[u].y * b[u].x);
                if (j < n12) X[j] = cmul(gg[u], t);
            }
        }
    } else {
        const ot* op = opl + E.opl_off + (ps * 12 + (f - R)) * nsig + (size_t)xpar * n12;
        for (int j0 = threadIdx.x; j0 < n12; j0 += 4 * blockDim.x) {
            ot v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = op[min(j0 + u * (int)blockDim.x, n12 - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j0 + u * (int)blockDim.x < n12) X[j0 + u * blockDim.x] = make_double2((double)v[u], 0.0);
        }
    }
    __syncthreads();
    double2* out = f < R ? sph + E.sph_off + (((size_t)id * Si + s) * R + f) * nsig + (size_t)xpar * n12
                         : spo + E.spo_off + (((size_t)id * Si + s) * 12 + (f - R)) * nsig + (size_t)xpar * n12;
    const FftPlan P1 = fft_plan(n1), P2 = fft_plan(n2);
    if (P1.n_st > 0 && P2.n_st > 0) {
        // along v (sequences u, contiguous), result left in X or Y, then along u
        // (sequences k2, stride n2), the last stage writing out[k1 n2 + k2]
        double2* mid = (P2.n_st & 1) ? Y : X;
        if constexpr (NP > 0) {
            if (n1 == NP && n2 == NP) {  // uniform for the block
                fft_axis_c<NP, 0>(X, Y, n2, 1, w2, sg, mid, n2, 1);
                fft_axis_c<NP, 0>(mid, mid == X ? Y : X, 1, n2, w1, sg, out, 1, n2);
                return;
            }
        }
        fft_axis(P2, X, Y, n2, 1, n2, n1, w2, sg, mid, n2, 1);
        fft_axis(P1, mid, mid == X ? Y : X, 1, n2, n1, n2, w1, sg, out, 1, n2);
        return;
    }
    // an extent with a prime factor above 5: direct sums (tiles of T x T outputs per thread)
    dft_axis<T>(X, n1, n2, n2, 1, w2, Y, n2, 1);
    __syncthreads();
    dft_axis<T>(Y, n2, n1, 1, n2, w1, out, 1, n2);
}

// ---------------------------------------------------------------------------
// Spectral sums of one measurement.  Work-group per (ensemble, axis, slab,
// probe group, run of kMacK values of k); the 12 O rows of those k for every
// x_par are staged in LDS once and shared by all separations r:
//   F[...][c][kind][g][k] += sum_{x_par} O^_{row}(x_par + l) (k) * h^~_r(x_par) (k)
// with l = l_g + (mode_g ? l_mid(r, c) : 0) and row = 2 o(c, axis) + kind.
// Work-item (k, r slot) takes r = slot, slot + kMacThreads / kMacK, ...  Every
// sum runs over x_par in ascending order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kMacThreads) k_spec_mac(const EnsDesc* __restrict__ ens,
                                                          const int* __restrict__ bstart, int n_ens,
                                                          const ObsDesc* __restrict__ obs,
                                                          const int* __restrict__ rlist, const int* __restrict__ comps,
                                                          const int* __restrict__ gdesc, const double2* __restrict__ sph,
                                                          const double2* __restrict__ spo, double2* __restrict__ facc)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double2* os = reinterpret_cast<double2*>(lds_raw);  // [row][x_par][kk]
    constexpr int KC = kMacK;
    const int e = find_ens_s(bstart, n_ens, blockIdx.x);
    const EnsDesc& E = ens[e];
    const ObsDesc& O = *obs;
    const int nsig = E.nsig, Si = E.s_in, R = O.n_r, Nc = O.n_comp, NG = O.n_groups;
    const int n3[3] = {E.nx, E.ny, E.nz};
    int n12max = 0;
    for (int i = 0; i < O.n_dirs; ++i) n12max = max(n12max, nsig / n3[O.dirs[i]]);
    const int nkc = (n12max + KC - 1) / KC;
    int local = blockIdx.x - bstart[e];
    const int kc = local % nkc;
    local /= nkc;
    const int g = local % NG;
    local /= NG;
    const int s = local % Si;
    const int id = local / Si;
    if (id >= O.n_dirs) return;
    const int dir = O.dirs[id];
    const int N = n3[dir], n12 = nsig / N;
    const int k0 = kc * KC;
    if (k0 >= n12) return;  // uniform for the block
    const size_t ps = (size_t)id * Si + s;
    // staged four elements per work-item and round, all loads issued before the LDS stores
    const int n_os = 12 * N * KC;
    for (int i0 = threadIdx.x; i0 < n_os; i0 += 4 * blockDim.x) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = min(i0 + u * (int)blockDim.x, n_os - 1);
            const int kk = i % KC, t = i / KC;
            const int xp = t % N, row = t / N;
            v[u] = k0 + kk < n12 ? spo[E.spo_off + (ps * 12 + row) * nsig + (size_t)xp * n12 + k0 + kk]
                                 : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * (int)blockDim.x < n_os) os[i0 + u * blockDim.x] = v[u];
    }
    __syncthreads();
    const int kk = threadIdx.x % KC, slot = threadIdx.x / KC;
    const int k = k0 + kk;
    if (k >= n12) return;
    for (int ir = slot; ir < R; ir += blockDim.x / KC) {
        const int r = rlist[ir];
        const double2* h = sph + E.sph_off + (ps * R + ir) * nsig + k;
        int xo[kMacComps], orow[kMacComps];
        double re[kMacComps][2], im[kMacComps][2];
#pragma unroll
        for (int ic = 0; ic < kMacComps; ++ic) {
            const int c = comps[ic < Nc ? ic : 0];
            const int l = gdesc[2 * g] + (gdesc[2 * g + 1] ? (spans_axis(c) ? (r - 1) / 2 : r / 2) : 0);
            xo[ic] = ((l % N) + N) % N;
            orow[ic] = 2 * orient_of(c, dir);
            re[ic][0] = im[ic][0] = re[ic][1] = im[ic][1] = 0.0;
        }
#pragma unroll 8
        for (int xp = 0; xp < N; ++xp) {
            const double2 b = h[(size_t)xp * n12];
#pragma unroll
            for (int ic = 0; ic < kMacComps; ++ic) {
                if (ic < Nc) {
#pragma unroll
                    for (int kind = 0; kind < 2; ++kind) {
                        const double2 a = os[((orow[ic] + kind) * N + xo[ic]) * KC + kk];
                        re[ic][kind] += a.x * b.x - a.y * b.y;
                        im[ic][kind] += a.x * b.y + a.y * b.x;
                    }
                    if (++xo[ic] == N) xo[ic] = 0;
                }
            }
        }
#pragma unroll
        for (int ic = 0; ic < kMacComps; ++ic) {
            if (ic < Nc) {
#pragma unroll
                for (int kind = 0; kind < 2; ++kind) {
                    const size_t sl = (((ps * R + ir) * Nc + ic) * 2 + kind) * NG + g;
                    double2* F = facc + E.facc_off + sl * n12max + k;
                    *F = make_double2(F->x + re[ic][kind], F->y + im[ic][kind]);
                }
            }
        }
    }
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
                       const double2* out_t, double scale, double2* wf, const double* results, const int* d_ring,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_wfac, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, out_t, scale, wf,
                       results, d_ring);
    return hipGetLastError();
}

hipError_t launch_gfac(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, const ObsDesc* d_obs,
                       const double2* avg_t, const double2* wf, int q, double2* gf, const double* results,
                       const int* d_ring, hipStream_t st)
{
    hipLaunchKernelGGL(k_gfac, dim3(total_blocks), dim3(256), 0, st, d_ens, d_bstart, n_ens, d_obs, avg_t, wf, q, gf,
                       results, d_ring);
    return hipGetLastError();
}

// tile: 4 when every transverse extent is a multiple of 4, else 2 (extents are even)
hipError_t launch_plane_stage(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks,
                              const ObsDesc* d_obs, const double2* hist_c, const void* hist_o, int m_in,
                              int precision, double2* cpl, void* opl, hipStream_t st)
{
    if (total_blocks <= 0) return hipSuccess;
    static_assert(kStageTile == 32, "the staging work-group is 32 x 8 threads");
    if (precision == 0)
        hipLaunchKernelGGL(k_plane_stage<double>, dim3(total_blocks), dim3(kStageTile * 8), 0, st, d_ens, d_bstart, n_ens, d_obs,
                           hist_c, (const double*)hist_o, m_in, cpl, (double*)opl);
    else
        hipLaunchKernelGGL(k_plane_stage<float>, dim3(total_blocks), dim3(kStageTile * 8), 0, st, d_ens, d_bstart, n_ens, d_obs,
                           hist_c, (const float*)hist_o, m_in, cpl, (float*)opl);
    return hipGetLastError();
}

hipError_t launch_dft_planes(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, size_t lds_bytes,
                             const ObsDesc* d_obs, const int* d_r, const double2* cpl, const void* opl,
                             const double2* gf, double2* sph, double2* spo, int precision, int tile,
                             hipStream_t st)
{
    const dim3 g(total_blocks), b(kPlaneThreads);
    // 48 x 48 planes (the 48^3 lattice) take the transform with constant sizes
    if (precision == 0) {
        if (tile == 4)
            hipLaunchKernelGGL((k_dft_planes<double, 4, 48>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               cpl, (const double*)opl, gf, sph, spo);
        else
            hipLaunchKernelGGL((k_dft_planes<double, 2, 0>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               cpl, (const double*)opl, gf, sph, spo);
    } else {
        if (tile == 4)
            hipLaunchKernelGGL((k_dft_planes<float, 4, 48>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               cpl, (const float*)opl, gf, sph, spo);
        else
            hipLaunchKernelGGL((k_dft_planes<float, 2, 0>), g, b, lds_bytes, st, d_ens, d_bstart, n_ens, d_obs, d_r,
                               cpl, (const float*)opl, gf, sph, spo);
    }
    return hipGetLastError();
}

hipError_t launch_spec_mac(const EnsDesc* d_ens, const int* d_bstart, int n_ens, int total_blocks, int npm,
                           const ObsDesc* d_obs, const int* d_r, const int* d_comp, const int* d_gdesc,
                           const double2* sph, const double2* spo, double2* facc, hipStream_t st)
{
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spec_mac, dim3(total_blocks), dim3(kMacThreads), spec_mac_lds(npm), st, d_ens, d_bstart,
                       n_ens, d_obs, d_r, d_comp, d_gdesc, sph, spo, facc);
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
