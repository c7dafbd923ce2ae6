// device_common.hpp -- device building blocks of libu1ml (gfx950).
//
// Link storage: one angle array per (ensemble, direction mu, parity), the
// sites of one parity packed along x: half index
//   h = (x >> 1) + (Nx/2) * (y + Ny * (z + Nz * t)),
// so consecutive work-items touch consecutive words for every neighbour
// (coalesced), and a checkerboard phase reads and writes whole cache lines.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace u1ml {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// -> 64 bit multiplications by fixed odd constants, with the Weyl-bumped key
// xored into the high halves.  Counter-based: no generator state in memory.
// ---------------------------------------------------------------------------
struct Block4 {
    uint32_t w[4];
};

// a ^ b ^ c in one instruction (gfx950 three-input bitwise op, truth table 0x96)
__device__ inline uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }

__device__ inline Block4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Block4 b;
    b.w[0] = c0;
    b.w[1] = c1;
    b.w[2] = c2;
    b.w[3] = c3;
    return b;
}

enum : uint32_t { DOM_HB = 0, DOM_INIT = 1, DOM_METRO = 2, DOM_TEST = 3 };

// ---------------------------------------------------------------------------
// FP32 atan2 without branches: octant reduction to q = min/max in [0, 1] and
// atan(q) = q P(q^2), P a degree-7 polynomial in q^2 fitted for this library
// (iteratively reweighted least squares towards the minimax fit on [0, 1]).
// Maximum error over the plane 3.2e-7 rad when evaluated in FP32.
// ---------------------------------------------------------------------------
__device__ inline float atan2_fast(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float q = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float s = q * q;
    float p = -0.004054566379636526f;
    p = fmaf(p, s, 0.021862950176000595f);
    p = fmaf(p, s, -0.055912312120199203f);
    p = fmaf(p, s, 0.09642195701599121f);
    p = fmaf(p, s, -0.1390862911939621f);
    p = fmaf(p, s, 0.19946564733982086f);
    p = fmaf(p, s, -0.33329859375953674f);
    p = fmaf(p, s, 0.9999993443489075f);
    float r = q * p;
    r = ay > ax ? 1.57079633f - r : r;
    r = x < 0.0f ? 3.14159265f - r : r;
    return copysignf(r, y);
}

// ---------------------------------------------------------------------------
// FP64 sine and cosine for |x| < 2^22, the arguments of this library (angle
// sums of a few links, pi u with u in (0, 1), slab sums of temporal links).
// Cody-Waite reduction x = q pi/2 + r, |r| <= pi/4 + tiny, with pi/2 split
// into three parts of which the first two carry 30 significant bits (q pi/2
// parts exact for |q| < 2^23, and x - q P1 exact by Sterbenz's lemma since
// x / (q P1) lies in [1/2, 2]); then sin r = r + r^3 S(r^2) and
// cos r = 1 - r^2/2 + r^4 C(r^2) (with 1 - r^2/2 carried as a rounded value
// plus its exact rounding error), S and C of degree 5 fitted for this library
// by a Remez exchange in 50-digit arithmetic (polynomial error below
// 1e-17 absolute on [-pi/4, pi/4]; what remains is FP64 rounding, about an
// ulp), and the quadrant q mod 4 selects and signs the pair.
// ---------------------------------------------------------------------------
__device__ inline void sincos_bounded(double x, double* sp, double* cp)
{
    const double q = rint(x * 0.63661977236758138);  // x * 2/pi
    double r = fma(-q, 1.570796325802803, x);         // pi/2, first 30 bits
    r = fma(-q, 9.920935791635221e-10, r);            // next 30 bits
    r = fma(-q, 5.170182981794105e-19, r);            // the rest
    const double z = r * r;
    double ps = 1.5918142569704652e-10;
    ps = fma(ps, z, -2.505113204972727e-08);
    ps = fma(ps, z, 2.7557316103657487e-06);
    ps = fma(ps, z, -0.00019841269836761008);
    ps = fma(ps, z, 0.00833333333333095);
    ps = fma(ps, z, -0.16666666666666666);
    const double s = fma(r * z, ps, r);
    double pc = -1.1382639805756885e-11;
    pc = fma(pc, z, 2.0876146382220145e-09);
    pc = fma(pc, z, -2.7557317272344146e-07);
    pc = fma(pc, z, 2.480158729876704e-05);
    pc = fma(pc, z, -0.0013888888888887398);
    pc = fma(pc, z, 0.041666666666666664);
    // cos: w = 1 - z/2 rounded, plus its rounding error (1 - w) - z/2, exact
    // by Sterbenz's lemma, so the sum keeps the low bits w dropped
    const double w = fma(-0.5, z, 1.0);
    const double c = w + fma(z * z, pc, (1.0 - w) - 0.5 * z);
    const int n = (int)q & 3;
    const double a = (n & 1) ? c : s;   // sine before the sign
    const double b = (n & 1) ? s : c;   // cosine before the sign
    *sp = (n & 2) ? -a : a;
    *cp = ((n + 1) & 2) ? -b : b;
}

// ---------------------------------------------------------------------------
// Precision traits.  FP64: the bounded sincos above where arguments are
// bounded, library math (ocml) otherwise, same formulas and order as the
// definitions; FP32: hardware transcendentals where the error budget allows.
// ---------------------------------------------------------------------------
template <typename real>
struct M;

template <>
struct M<double> {
    static constexpr double pi = 3.141592653589793;
    static constexpr double two_pi = 6.283185307179586;
    __device__ static inline void sincos_(double a, double* s, double* c) { sincos_bounded(a, s, c); }
    __device__ static inline double cos_pi(double u)  // cos(pi u), 0 < u < 1
    {
        double s, c;
        sincos_bounded(pi * u, &s, &c);
        return c;
    }
    __device__ static inline double atan2_(double y, double x) { return atan2(y, x); }
    __device__ static inline double acos_(double x) { return acos(x); }
    __device__ static inline double log_(double x) { return log(x); }
    __device__ static inline double exp_(double x) { return exp(x); }
    __device__ static inline double sqrt_(double x) { return sqrt(x); }
    __device__ static inline double div_(double a, double b) { return a / b; }
    __device__ static inline double floor_(double x) { return floor(x); }
    // U1 from the high 31 bits of word a, U2 from the whole word b, in (0, 1)
    __device__ static inline double u1(uint32_t a) { return ((double)(a >> 1) + 0.5) * (1.0 / 2147483648.0); }
    __device__ static inline double u2(uint32_t b) { return ((double)b + 0.5) * (1.0 / 4294967296.0); }
};

template <>
struct M<float> {
    static constexpr float pi = 3.14159265f;
    static constexpr float two_pi = 6.28318531f;
    // hardware sin/cos take revolutions; |a| < 4 pi here, well inside their range
    __device__ static inline void sincos_(float a, float* s, float* c)
    {
        const float rev = a * 0.159154943f;
        *s = __builtin_amdgcn_sinf(rev);
        *c = __builtin_amdgcn_cosf(rev);
    }
    __device__ static inline float cos_pi(float u) { return __builtin_amdgcn_cosf(0.5f * u); }
    __device__ static inline float atan2_(float y, float x) { return atan2_fast(y, x); }
    __device__ static inline float acos_(float x) { return acosf(x); }
    __device__ static inline float log_(float x) { return __logf(x); }
    __device__ static inline float exp_(float x) { return __expf(x); }
    // hardware square root (1 ulp), without the correctly rounded library's refinement
    __device__ static inline float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static inline float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    __device__ static inline float floor_(float x) { return floorf(x); }
    // 23-bit uniforms: exact in FP32, never 0 or 1
    __device__ static inline float u1(uint32_t a) { return ((float)(a >> 9) + 0.5f) * (1.0f / 8388608.0f); }
    __device__ static inline float u2(uint32_t b) { return ((float)(b >> 9) + 0.5f) * (1.0f / 8388608.0f); }
};

// wrap(a) = a - 2 pi floor((a + pi) / (2 pi))
template <typename real>
__device__ inline real wrap_angle(real a)
{
    return a - M<real>::two_pi * M<real>::floor_((a + M<real>::pi) / M<real>::two_pi);
}

template <>
__device__ inline float wrap_angle<float>(float a)
{
    return a - 6.28318531f * floorf(fmaf(a, 0.159154943f, 0.5f));
}

// ---------------------------------------------------------------------------
// von Mises(0, kappa) by Best & Fisher (1979): wrapped-Cauchy envelope with
//   s = sqrt(1 + 4 k^2), tau = 1 + s, rho = 2 k tau / ((s+1)(tau + sqrt(2 tau)))
//   (the cancellation-free form of (tau - sqrt(2 tau)) / (2 k)),
//   r = (1 + rho^2) / (2 rho);
// attempt: z = cos(pi U1), f = (1 + r z)/(r + z), c = k (r - f), accept if
// c (2 - c) > U2 or ln(c / U2) + 1 - c >= 0; psi = sign * arccos(f).
// Attempt j reads Philox block (c0, c1, j/2, domain): words (0,1) for even j,
// (2,3) for odd j; sign = low bit of the first word of the pair.
// Returns psi and the attempt count (-1 past 65536 attempts).
// ---------------------------------------------------------------------------
template <typename real>
__device__ inline real vonmises_psi(real kappa, uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t domain,
                                    int* n_att);

// The envelope parameter r and one Philox block's two attempts (2j from words
// 0, 1 and 2j+1 from words 2, 3) in FP64; the pair returns which attempt
// accepted first (1 or 2, with its psi) or 0.
__device__ inline double bf_r_f64(double kappa)
{
    using m = M<double>;
    const double s = m::sqrt_(1.0 + 4.0 * kappa * kappa);
    const double tau = 1.0 + s;
    const double rho = m::div_(2.0 * kappa * tau, (s + 1.0) * (tau + m::sqrt_(2.0 * tau)));
    return m::div_(1.0 + rho * rho, 2.0 * rho);
}

// Both attempts are evaluated by every lane, so a wave runs each step once
// whichever attempt its lanes accept; the accepted attempt is returned as
// cos(psi) = f and the sign of psi (psi = -arccos f when negative).
// The logarithmic test is decided on t = ln(c / U2) + 1 - c formed in FP32
// (hardware base-2 logarithm): with 1/2 <= c < 64 and U2 >= 2^-33,
// |ln(c / U2)| < 28 and the FP32 value is within 1e-5 of the exact one; where
// |t| < 2^-10, or c >= 64 (kappa above 31), the test is taken again in FP64
// exactly as the definition writes it.  Every decision is the FP64 test's.
__device__ inline int bf_pair_f64(double kappa, double r, const Block4& b, double* cpsi, bool* neg)
{
    using m = M<double>;
    double f[2], c[2], u2[2];
    bool acc[2], band[2];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const uint32_t a = half ? b.w[2] : b.w[0];
        const uint32_t bb = half ? b.w[3] : b.w[1];
        const double z = m::cos_pi(m::u1(a));
        double fh = m::div_(1.0 + r * z, r + z);
        fh = fh > 1.0 ? 1.0 : (fh < -1.0 ? -1.0 : fh);
        f[half] = fh;
        c[half] = kappa * (r - fh);
        u2[half] = m::u2(bb);
        const bool quick = c[half] * (2.0 - c[half]) - u2[half] > 0.0;
        const float t = fmaf(__builtin_amdgcn_logf((float)c[half] * __builtin_amdgcn_rcpf((float)u2[half])),
                             0.693147181f, (float)(1.0 - c[half]));
        acc[half] = quick || t >= 0.0f;
        band[half] = !quick && (fabsf(t) < 0.0009765625f || c[half] >= 64.0);
    }
    if (band[0] || band[1]) {
#pragma unroll
        for (int half = 0; half < 2; ++half)
            if (band[half]) acc[half] = m::log_(m::div_(c[half], u2[half])) + 1.0 - c[half] >= 0.0;
    }
    if (!acc[0] && !acc[1]) return 0;
    *cpsi = acc[0] ? f[0] : f[1];
    *neg = ((acc[0] ? b.w[0] : b.w[2]) & 1u) != 0;
    return acc[0] ? 1 : 2;
}

template <>
__device__ inline double vonmises_psi<double>(double kappa, uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                              uint32_t domain, int* n_att)
{
    using m = M<double>;
    if (kappa == 0.0) {
        const Block4 b = philox4x32_10(c0, c1, 0u, domain, k0, k1);
        *n_att = 1;
        return m::pi * (2.0 * m::u1(b.w[0]) - 1.0);
    }
    const double r = bf_r_f64(kappa);
    for (uint32_t jp = 0; jp < 32768u; ++jp) {
        double f;
        bool neg;
        const int k = bf_pair_f64(kappa, r, philox4x32_10(c0, c1, jp, domain, k0, k1), &f, &neg);
        if (k) {
            *n_att = 2 * (int)jp + k;
            const double p = m::acos_(f);
            return neg ? -p : p;
        }
    }
    *n_att = -1;
    return 0.0;
}

// FP32 form of the same sampler.  With s = sqrt(1 + 4 kappa^2), Best and
// Fisher's rho and r = (1 + rho^2) / (2 rho) reduce to r = (1 + s) / (2 kappa)
// (1 / rho = (tau + sqrt(2 tau)) / (2 kappa) because tau (tau - 2) = 4 kappa^2),
// and since s - 2 kappa = 1 / (s + 2 kappa),
//   r - 1 = (1 + 1 / (s + 2 kappa)) / (2 kappa)
// without cancellation at any kappa.  An attempt is rewritten so that small
// |psi| (f near 1) and |psi| near pi (f near -1) keep their relative
// precision: with a = pi U1 / 2, 1 - z = 2 sin^2 a, 1 + z = 2 cos^2 a and
//   g = 1 - f = (r - 1)(1 - z) / (r + z) = (r - 1) sin^2 a / ((r - 1) / 2 + cos^2 a),
//   h = 1 + f = (r + 1)(1 + z) / (r + z) = (r + 1) cos^2 a / ((r - 1) / 2 + cos^2 a),
//   c = kappa (r - f) = kappa (r - 1) + kappa g,
// the same quantities as above.  Since kappa (r - 1) = (1 + s - 2 kappa) / 2
// >= 1/2, c >= 1/2 and c / U2 is a normal number, so the logarithmic test
// ln(c / U2) + 1 - c >= 0 is taken in base 2 on the hardware logarithm:
// log2(c / U2) >= (c - 1) log2(e).  An accepted deviate is returned as
// cos(psi) = 1 - g (or h - 1 when g > 1) and sin(psi) = sign sqrt(g h).
struct BfEnvF32 {
    float kappa, rm1, half_rm1, rp1, krm1;  // kappa, r - 1, (r - 1) / 2, r + 1, kappa (r - 1)
};

__device__ inline BfEnvF32 bf_env_f32(float kappa)
{
    const float s = __builtin_amdgcn_sqrtf(fmaf(4.0f * kappa, kappa, 1.0f));
    const float rm1 = (1.0f + __builtin_amdgcn_rcpf(fmaf(2.0f, kappa, s))) * (0.5f * __builtin_amdgcn_rcpf(kappa));
    return BfEnvF32{kappa, rm1, 0.5f * rm1, rm1 + 2.0f, kappa * rm1};
}

// Attempts 2j and 2j+1 of the block b (words 0, 1 then 2, 3); returns which
// accepted first (1 or 2, with (cos psi, sin psi) of that attempt) or 0.
__device__ inline int bf_pair_f32(const BfEnvF32& v, const Block4& b, float* cpsi, float* spsi)
{
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const uint32_t a = half ? b.w[2] : b.w[0];
        const uint32_t bb = half ? b.w[3] : b.w[1];
        // pi U1 / 2 in revolutions, U1 = ((a >> 9) + 1/2) 2^-23 (exact)
        const float q = fmaf((float)(a >> 9), 1.0f / 33554432.0f, 1.0f / 67108864.0f);
        const float sh = __builtin_amdgcn_sinf(q), ch = __builtin_amdgcn_cosf(q);
        const float sh2 = sh * sh, ch2 = ch * ch;
        const float inv = __builtin_amdgcn_rcpf(v.half_rm1 + ch2);
        const float g = v.rm1 * sh2 * inv;
        const float c = fmaf(v.kappa, g, v.krm1);
        const float u2 = fmaf((float)(bb >> 9), 1.0f / 8388608.0f, 1.0f / 16777216.0f);
        bool acc = c * (2.0f - c) - u2 > 0.0f;
        if (!acc) acc = __builtin_amdgcn_logf(c * __builtin_amdgcn_rcpf(u2)) >= (c - 1.0f) * 1.44269504f;
        if (acc) {
            const float h = v.rp1 * ch2 * inv;
            const float sp = __builtin_amdgcn_sqrtf(g * h);
            *cpsi = g <= 1.0f ? 1.0f - g : h - 1.0f;
            *spsi = __uint_as_float(__float_as_uint(sp) ^ (a << 31));
            return half + 1;
        }
    }
    return 0;
}

__device__ inline void vonmises_cs_f32(float kappa, uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t domain,
                                       float* cpsi, float* spsi, int* n_att)
{
    if (kappa == 0.0f) {
        const Block4 b = philox4x32_10(c0, c1, 0u, domain, k0, k1);
        const float rev = M<float>::u1(b.w[0]) - 0.5f;  // psi = pi (2 U1 - 1) in revolutions
        *cpsi = __builtin_amdgcn_cosf(rev);
        *spsi = __builtin_amdgcn_sinf(rev);
        *n_att = 1;
        return;
    }
    const BfEnvF32 v = bf_env_f32(kappa);
    for (uint32_t jp = 0; jp < 32768u; ++jp) {
        const Block4 b = philox4x32_10(c0, c1, jp, domain, k0, k1);
        float cp, sp;
        const int k = bf_pair_f32(v, b, &cp, &sp);
        if (k) {
            *n_att = 2 * (int)jp + k;
            *cpsi = cp;
            *spsi = sp;
            return;
        }
    }
    *n_att = -1;
    *cpsi = 1.0f;
    *spsi = 0.0f;
}

template <>
__device__ inline float vonmises_psi<float>(float kappa, uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                            uint32_t domain, int* n_att)
{
    float cp, sp;
    vonmises_cs_f32(kappa, k0, k1, c0, c1, domain, &cp, &sp, n_att);
    return atan2_fast(sp, cp);
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
struct Coord {
    int x, y, z, t;
};

__device__ inline int wrap_p(int v, int n) { return v == n ? 0 : v; }
__device__ inline int wrap_m(int v, int n) { return v < 0 ? n - 1 : v; }

__device__ inline Coord step(Coord c, int dir, int s, int nx, int ny, int nz, int nt)
{
    switch (dir) {
    case 0: c.x = s > 0 ? wrap_p(c.x + 1, nx) : wrap_m(c.x - 1, nx); break;
    case 1: c.y = s > 0 ? wrap_p(c.y + 1, ny) : wrap_m(c.y - 1, ny); break;
    case 2: c.z = s > 0 ? wrap_p(c.z + 1, nz) : wrap_m(c.z - 1, nz); break;
    default: c.t = s > 0 ? wrap_p(c.t + 1, nt) : wrap_m(c.t - 1, nt); break;
    }
    return c;
}

// ---------------------------------------------------------------------------
// Division-free index decode: q = a / b for 0 <= a < 2^31, 0 < b < 2^24
// (the correction multiplies in 24 bits) and a / b < 2^22, from the FP32
// reciprocal and one exact correction step.
// ---------------------------------------------------------------------------
__device__ inline int fdiv(int a, int b, float inv_b)
{
    int q = (int)((float)a * inv_b);
    const int r = a - (int)__umul24(q, b);
    q += (r >= b) - (r < 0);
    return q;
}

// Site in even/odd storage: coordinates and hrow = (Nx/2) (y + Ny (z + Nz t)),
// so the half index of a site is (x >> 1) + hrow.
struct Site {
    int x, y, z, t, hrow;
};

struct Geo {
    int nx, ny, nz, nt, sy, sz, st;  // sy = Nx/2, sz = sy Ny, st = sz Nz (strides in half indices)
};

// one periodic step along compile-time direction D, sign S.  The wrap is
// written with an all-ones mask w (= -1 when the step crosses the boundary),
// so the step is a few integer operations with no branch.
template <int D, int S>
__device__ inline Site mv(Site c, const Geo& g)
{
    if (D == 0) {
        const int w = -(int)(S > 0 ? c.x == g.nx - 1 : c.x == 0);
        c.x = S > 0 ? (c.x + 1) & ~w : c.x - 1 + (w & g.nx);
        return c;
    }
    const int n = D == 1 ? g.ny : D == 2 ? g.nz : g.nt;
    const int st = D == 1 ? g.sy : D == 2 ? g.sz : g.st;
    int& v = D == 1 ? c.y : D == 2 ? c.z : c.t;
    const int w = -(int)(S > 0 ? v == n - 1 : v == 0);
    if (S > 0) {
        c.hrow += st - (w & (n * st));
        v = (v + 1) & ~w;
    } else {
        c.hrow += (w & (n * st)) - st;
        v = v - 1 + (w & n);
    }
    return c;
}

__device__ inline unsigned hidx(const Site& c) { return (unsigned)((c.x >> 1) + c.hrow); }

// Load from a uniform base with a 32-bit byte offset (one ensemble's links
// span less than 4 GiB), which maps to global_load with a scalar base.
template <typename real>
__device__ inline real ldo(const real* __restrict__ base, unsigned byte_off)
{
    return *reinterpret_cast<const real*>(reinterpret_cast<const char*>(base) + byte_off);
}

// ---------------------------------------------------------------------------
// Staple gathers (links as even/odd arrays of angles, see ldo / hidx)
// ---------------------------------------------------------------------------
// The six angles of the two staples of link (x, MU) in the plane (MU, NU):
//   v[0..2] = th_nu(x+mu), th_mu(x+nu), th_nu(x)          (forward)
//   v[3..5] = th_nu(x-nu), th_nu(x+mu-nu), th_mu(x-nu)    (backward)
// The angles of direction d and parity par start at element (2 d + par) vh.
template <typename real, int MU, int NU>
__device__ inline void gather_plane(const real* __restrict__ lb, unsigned vh, const Geo& g, const Site& c,
                                    const Site& cpm, int p, real* v)
{
    const unsigned q = p ^ 1;
    const Site cpn = mv<NU, +1>(c, g);
    const Site cmn = mv<NU, -1>(c, g);
    const Site cpmmn = mv<NU, -1>(cpm, g);
    constexpr unsigned w = sizeof(real);
    v[0] = ldo(lb, ((NU * 2 + q) * vh + hidx(cpm)) * w);
    v[1] = ldo(lb, ((MU * 2 + q) * vh + hidx(cpn)) * w);
    v[2] = ldo(lb, ((NU * 2 + p) * vh + hidx(c)) * w);
    v[3] = ldo(lb, ((NU * 2 + q) * vh + hidx(cmn)) * w);
    v[4] = ldo(lb, ((NU * 2 + p) * vh + hidx(cpmmn)) * w);
    v[5] = ldo(lb, ((MU * 2 + q) * vh + hidx(cmn)) * w);
}

template <int MU, int K>
struct Nu {  // K-th direction other than MU, ascending
    static constexpr int v = K < MU ? K : K + 1;
};


// Staple sum A = sum_{nu != MU} exp(i phi_f) + exp(i phi_b), nu ascending,
// forward before backward, of the link (c, MU) of parity p (cpm = c + MU).
template <typename real, int MU>
__device__ inline void staple_sum(const real* __restrict__ lb, unsigned vh, const Geo& g, const Site& c,
                                  int p, real* ar, real* ai)
{
    const Site cpm = mv<MU, +1>(c, g);
    real v[3][6];
    gather_plane<real, MU, Nu<MU, 0>::v>(lb, vh, g, c, cpm, p, v[0]);
    gather_plane<real, MU, Nu<MU, 1>::v>(lb, vh, g, c, cpm, p, v[1]);
    gather_plane<real, MU, Nu<MU, 2>::v>(lb, vh, g, c, cpm, p, v[2]);
    real sr = real(0), si = real(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        real s, co;
        M<real>::sincos_(v[k][0] - v[k][1] - v[k][2], &s, &co);
        sr += co;
        si += s;
        M<real>::sincos_(v[k][3] - v[k][4] - v[k][5], &s, &co);
        sr += co;
        si += s;
    }
    *ar = sr;
    *ai = si;
}

// I_1(k) / I_0(k) from the ratio recurrence I_{n-1}/I_n = 2n/k + I_{n+1}/I_n
// (continued fraction 1/(2/k + 1/(4/k + ...))), evaluated backwards from
// depth 40 + ceil(k); relative error below 1e-15 for k <= 100.
__device__ inline double bessel_ratio(double k)
{
    if (!(k > 0.0)) return 0.0;
    const int depth = 40 + (int)ceil(fmin(k, 4000.0));
    double t = 0.0;
    for (int n = depth; n >= 1; --n) t = 1.0 / (2.0 * n / k + t);
    return t;
}

}  // namespace u1ml
