// Tersoff energy / force / virial evaluation (Eq. 1-3, Algorithm 1) on the
// resident neighbour list, in three launches:
//
//   k_pack      skin exclusion and packing (Sections 2 and 3): every list
//               entry gets its FP64 minimum-image displacement and r^2; the
//               entries inside the interaction range become compact per-atom
//               records (displacement, membership bits).
//   k_tersoff   zeta, b_ij, energy, forces and virial from the records, one
//               wavefront per batch of centre atoms, one lane per pair (i, j).
//   k_gather_forces
//               F_m = (terms of centre m) + (terms of every centre i that
//               keeps m, stored in the force plane m reserved for i).
//
// `real` is float for the mixed path and double for the all-FP64 path; the
// displacement, the zeta -> b power (in the mixed path through the short
// FP64 log and exp of bond_order_f64) and every accumulation are FP64 in both.
// Each pair's force term on its neighbour is stored in the working precision
// (float planes for the mixed path) and summed per atom in FP64.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>

namespace tsf {

namespace {

// ---------------------------------------------------------------- math ----

template <typename real>
struct M;

template <>
struct M<float> {
    static __device__ __forceinline__ float exp(float x) { return expf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
};

template <>
struct M<double> {
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
};

// Minimum-image component: s = rint(t / L) evaluated as rint(t * (1/L)).
// For any pair within the interaction range t/L is far from a half-integer
// (the box is at least twice the list radius), so s -- and therefore d and
// r^2 -- equal the values of the division form bit for bit.
__device__ __forceinline__ double image(double t, double L, double invL)
{
#pragma clang fp contract(off)
    double s = rint(t * invL);
    return fma(-s, L, t);
}

__device__ __forceinline__ double norm2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// ---- FP64 logarithm and exponential of the zeta -> b power (Eq. 2) ----
//
// ln 2 split into a head with 21 significant bits (so k * head is exact for
// |k| < 2^11) and the rest.
constexpr double kLn2Hi = 0x1.62e42p-1;
constexpr double kLn2Lo = 0x1.fdf473de6af28p-22;
constexpr double kLog2e = 1.4426950408889634;

// 1/d in FP64: the hardware reciprocal estimate (at least 23 correct bits)
// and one Newton step (relative error below 2^-46 + rounding).
__device__ __forceinline__ double recip_f64(double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    return fma(fma(-d, r, 1.0), r, r);
}

// The mixed path's power needs b to about 1e-9 relative: zeta arrives as an
// FP32 sum (relative error ~1e-7), which already moves b by up to
// x / (2 (1 + x)) * 1e-7, and 1e-9 of b is ~4e-9 eV per pair.  The series
// below are cut where their truncation falls under that.
//
// Natural logarithm of y > 0 (+inf and NaN pass through): y = 2^e m with m in
// [1/sqrt 2, sqrt 2), ln m = 2 atanh(s), s = (m - 1) / (m + 1), |s| < 0.172,
// summed as 2 s sum_{k <= 4} s^(2k) / (2k + 1) (the first omitted term,
// 2 s^11 / 11, is below 7e-10), plus e ln 2 in two parts.
__device__ __forceinline__ double ln_f64(double y)
{
    if (!(y < INFINITY)) return y;
    double m = __builtin_amdgcn_frexp_mant(y);   // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(y);
    if (m < 0.7071067811865476) {
        m += m;
        e -= 1;
    }
    const double f = m - 1.0;                    // exact
    const double s = f * recip_f64(2.0 + f);
    const double s2 = s * s;
    double p = 1.0 / 9.0;
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double t = s + s;
    const double lnm = fma(t, s2 * p, t);
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, lnm));
}

// e^t: t = k ln 2 + r with k = rint(t / ln 2), |r| <= ln 2 / 2, e^r from its
// Taylor series through r^8 (truncation below 2.1e-10 relative), scaled by
// 2^k.  t is clamped to [-760, 760], beyond which the result is 0 or +inf.
__device__ __forceinline__ double exp_f64(double t)
{
    t = fmin(fmax(t, -760.0), 760.0);
    const double kf = rint(t * kLog2e);
    double r = fma(-kf, kLn2Hi, t);
    r = fma(-kf, kLn2Lo, r);
    double p = 1.0 / 40320.0;                   // 1/8!
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)kf);
}

// b(zeta) and db/dzeta of Eq. (2) in log form, zeta > 0 (mixed path; relative
// error of b a few 1e-9, a third of the instructions of the library
// functions):
// x = exp(eta (ln beta + ln zeta)), b = exp(-ln(1 + x) / (2 eta)),
// db/dzeta = -(1/2) b x / (zeta (1 + x)).
__device__ __forceinline__ void bond_order_f64(const ParamX &px, double zeta, double &b, double &db)
{
    const double x = exp_f64(px.eta * (px.logbeta + ln_f64(zeta)));
    const double y = 1.0 + x;
    b = exp_f64(-ln_f64(y) * px.inv2eta);
    db = -0.5 * b * x * recip_f64(zeta * y);
}

// r^2 of a packed displacement in the working precision (the FP64 form is
// the packing kernel's, so r is the same there)
__device__ __forceinline__ double norm2r(double dx, double dy, double dz) { return norm2(dx, dy, dz); }
__device__ __forceinline__ float norm2r(float dx, float dy, float dz) { return fmaf(dz, dz, fmaf(dy, dy, dx * dx)); }

// Largest a in [0, nseg) with starts[a] <= v (starts ascending, starts[0] <= v).
__device__ __forceinline__ int find_seg(const int *starts, int nseg, int v)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int lanes_below(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int u = __shfl_up(v, off, kWave);
        if (lane >= off) v += u;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

constexpr double inv_factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return 1.0 / f;
}

// ------------------------------------------------------------ parameters --

template <typename real>
__device__ __forceinline__ const ParamR<real> *table_r(const DeviceTable &t);
template <>
__device__ __forceinline__ const ParamR<float> *table_r<float>(const DeviceTable &t) { return t.pf; }
template <>
__device__ __forceinline__ const ParamR<double> *table_r<double>(const DeviceTable &t) { return t.pd; }

// e^(a + a_lo) for |a_lo| <= ulp(a) and |a| <= 80, from FP32 operations,
// returned in FP64 with a relative error near 2^-27 (an emulation of these
// steps in exactly rounded float arithmetic measures 0.13 float ulp).
// k = rint(a / ln 2); the reduced argument t = a - k ln 2 is kept as an
// unevaluated float pair (ln 2 split into a 17-bit head, so that k * head is
// exact, and a float tail; two-product and two-sum give the rounding
// errors); e^t = 1 + t + t^2 q(t), q the Taylor series of (e^t - 1 - t) / t^2
// through its t^6 term (truncation below 3e-10 on |t| <= ln 2 / 2), with
// 1 + t as an exact pair and every smaller term summed into its tail.
__device__ __forceinline__ void exp_pair_parts(float a, float a_lo, float &hi, float &lo, int &k)
{
#pragma clang fp contract(off)
    constexpr float kLog2eF = 1.44269504f;
    constexpr float kLn2HiF = 0x1.62e4p-1f;
    constexpr float kLn2LoF = (float)(0.69314718055994530942 - (double)0x1.62e4p-1f);
    const float kf = rintf(a * kLog2eF);
    const float t1 = fmaf(-kf, kLn2HiF, a);      // exact
    const float p = kf * kLn2LoF;
    const float pe = fmaf(kf, kLn2LoF, -p);      // kf * kLn2LoF = p + pe
    const float th = t1 - p;                     // two-sum of t1 and -p
    const float bb = th - t1;
    const float e1 = (t1 - (th - bb)) + (-p - bb);
    const float tl = (e1 - pe) + a_lo;           // a - k ln 2 = th + tl
    const float sq = th * th;
    const float sqe = fmaf(th, th, -sq);         // th^2 = sq + sqe
    float q = (float)inv_factorial(8);
    q = fmaf(q, th, (float)inv_factorial(7));
    q = fmaf(q, th, (float)inv_factorial(6));
    q = fmaf(q, th, (float)inv_factorial(5));
    q = fmaf(q, th, (float)inv_factorial(4));
    q = fmaf(q, th, (float)inv_factorial(3));
    q = fmaf(q, th, 0.5f);
    const float eth = 1.0f + fmaf(sq, q, th);    // e^th to about one ulp (weights tl only)
    const float tail = fmaf(tl, eth, fmaf(sq, q, sqe * q));
    hi = 1.0f + th;
    lo = ((1.0f - hi) + th) + tail;              // 1 + th = hi + ((1 - hi) + th) exactly
    k = (int)kf;
}

// The value 2^k (hi + lo) rounded once to float (the all-FP32 path).
__device__ __forceinline__ float exp_pair_f32_rounded(float a, float a_lo)
{
    float hi, lo;
    int k;
    exp_pair_parts(a, a_lo, hi, lo, k);
    return __builtin_amdgcn_ldexpf(hi + lo, k);
}

// The argument ln A - lambda r of A exp(-lambda r) as a float pair s + lo
// (all-FP32 path), for r = r + r_lo (FP64 distance as an unevaluated float
// pair), ln A = lnA + lnA_lo, lambda = l + l_lo (two-product, two-sum).
__device__ __forceinline__ void scaled_arg(float lnA, float lnA_lo, float l, float l_lo, float r, float r_lo,
                                           float &s, float &lo)
{
#pragma clang fp contract(off)
    const float p = l * r;
    const float pe = fmaf(l, r, -p);
    s = lnA - p;
    const float bb = s - lnA;
    const float e = (lnA - (s - bb)) + (-p - bb);
    lo = (((e + lnA_lo) - pe) - l_lo * r) - l * r_lo;
}

// A exp(-lambda r) for the FP64 distance r + r_lo given as a float pair and
// lambda = l + l_lo (mixed path), from FP32 operations: k = rint(-l r / ln 2);
// t = -l r - k ln 2 is kept as th + tl, th = -p - k head exact (p = RN(l r),
// the 17-bit head of ln 2 times k exact, Sterbenz) and tl the small rest
// (|tl| < 2e-5: the rounding error of l r, the lo parts of lambda and r, and
// k times the tail of ln 2); e^th (1 + tl) as in exp_pair_parts; the result
// 2^k (hi + lo) A in FP64.  Relative error near 2^-27 (an emulation of these
// steps in exactly rounded float arithmetic measures 0.13 float ulp).
__device__ __forceinline__ double exp_decay_f32(double A, float l, float l_lo, float r, float r_lo)
{
#pragma clang fp contract(off)
    constexpr float kLog2eF = 1.44269504f;
    constexpr float kLn2HiF = 0x1.62e4p-1f;
    constexpr float kLn2LoF = (float)(0.69314718055994530942 - (double)0x1.62e4p-1f);
    const float p = l * r;
    const float pe = fmaf(l, r, -p);             // l r = p + pe exactly
    const float kf = rintf(-p * kLog2eF);
    const float th = fmaf(kf, -kLn2HiF, -p);     // exact
    const float tl = (((-pe) - l_lo * r) - l * r_lo) - kf * kLn2LoF;
    const float sq = th * th;
    const float sqe = fmaf(th, th, -sq);         // th^2 = sq + sqe
    float q = (float)inv_factorial(8);
    q = fmaf(q, th, (float)inv_factorial(7));
    q = fmaf(q, th, (float)inv_factorial(6));
    q = fmaf(q, th, (float)inv_factorial(5));
    q = fmaf(q, th, (float)inv_factorial(4));
    q = fmaf(q, th, (float)inv_factorial(3));
    q = fmaf(q, th, 0.5f);
    const float eth = 1.0f + fmaf(sq, q, th);    // e^th to about one ulp (weights tl only)
    const float tail = fmaf(tl, eth, fmaf(sq, q, sqe * q));
    const float hi = 1.0f + th;
    const float lo = ((1.0f - hi) + th) + tail;  // 1 + th = hi + ((1 - hi) + th) exactly
    return __builtin_amdgcn_ldexp((double)hi + (double)lo, (int)kf) * A;
}

// f_R = A exp(-lambda1 r), f_A = -B exp(-lambda2 r) and their derivatives
// in the all-FP32 path: the exponentials of exp_pair_parts rounded once to
// float (the mixed path takes them in FP64, and the FP64 path evaluates
// them directly).
__device__ __forceinline__ void pair_terms(const ParamR<float> &q, float r, float &fr, float &dfr,
                                           float &fa, float &dfa, float r_lo = 0.f)
{
    float s, lo;
    scaled_arg(q.lnA, q.lnA_lo, q.lam1, q.lam1_lo, r, r_lo, s, lo);
    fr = exp_pair_f32_rounded(s, lo);
    scaled_arg(q.lnB, q.lnB_lo, q.lam2, q.lam2_lo, r, r_lo, s, lo);
    fa = -exp_pair_f32_rounded(s, lo);
    dfr = -fmaf(q.lam1, fr, q.lam1_lo * fr);
    dfa = -fmaf(q.lam2, fa, q.lam2_lo * fa);
}

__device__ __forceinline__ void pair_terms(const ParamR<double> &q, double r, double &fr,
                                           double &dfr, double &fa, double &dfa)
{
    fr = q.A * ::exp(-q.lam1 * r);
    fa = -q.B * ::exp(-q.lam2 * r);
    dfr = -q.lam1 * fr;
    dfa = -q.lam2 * fa;
}

// sin x and cos x for |x| <= pi/2 (the switching-function argument never
// leaves that interval, up to rounding) from their Taylor series, by Horner's
// rule in x^2: sin through the x^13 term and cos through x^14 in float
// (truncation below 7e-10 on the interval), through x^23 and x^24 in double
// (below 1e-20).  The general range reduction of the library routines,
// several times longer than the polynomials, is not needed.
template <typename real>
__device__ __forceinline__ void sincos_halfpi(real x, real &s, real &c)
{
    constexpr int K = sizeof(real) == 4 ? 6 : 11;   // sin: terms k = 0..K of (-1)^k x^(2k+1) / (2k+1)!
    const real z = x * x;
    real ps = real((K & 1 ? -1.0 : 1.0) * inv_factorial(2 * K + 1));
    real pc = real(((K + 1) & 1 ? -1.0 : 1.0) * inv_factorial(2 * K + 2));   // cos: k = 0..K+1
#pragma unroll
    for (int k = K; k >= 1; --k) {
        ps = ps * z + real((k & 1 ? 1.0 : -1.0) * inv_factorial(2 * k - 1));
        pc = pc * z + real((k & 1 ? -1.0 : 1.0) * inv_factorial(2 * k));
    }
    pc = pc * z + real(1);
    s = x * ps;
    c = pc;
}

// Switching function f_C(r) = 1/2 - 1/2 sin(pi/2 (r - R)/D) and its
// derivative, evaluated in the zone as sin^2(y), y = (pi/4)(R + D - r)/D --
// the same function without the cancellation of 1/2 - 1/2 sin(x) as x nears
// pi/2: near the cutoff f_C of a third atom k is tiny, yet the bond order's
// b'(zeta) ~ zeta^(eta - 1) keeps dV/dzeta dzeta/dx_k finite, so f_C needs
// its relative accuracy there (1/2 - 1/2 sin rounds to 0 in FP32 within
// 1e-4 A of the cutoff).  R + D - r is exact (Sterbenz), and the rounding
// errors of r (r_lo: the FP64 distance minus the working-precision one),
// R + D and pi/(4D) are added back.
template <typename real>
__device__ __forceinline__ void cutoff_terms(const ParamR<real> &q, real r, real &fc, real &dfc, real r_lo = real(0))
{
    fc = real(1);
    dfc = real(0);
    if (r >= q.Rin) {
        const real dr = (q.Rc - r) + (q.Rc_lo - r_lo);
        const real y = dr * q.qpi_D + dr * q.qpi_D_lo;
        real sn, cn;
        sincos_halfpi(y, sn, cn);
        fc = sn * sn;
        dfc = real(-2) * (q.qpi_D + q.qpi_D_lo) * sn * cn;
    }
}

// -------------------------------------------------------- packed records -

// One packed neighbour n of a centre atom i (an in-range entry of i's list,
// Section 3): one word with the neighbour index, its type and the
// membership bits of the exact FP64 cutoff tests, and the minimum-image
// displacement in the working precision (distance and unit vector are formed
// from it by the compute kernel) -- 16 bytes (one vector load) for the
// single-precision displacement, 32 for FP64.  The records of a batch of B
// consecutive centre atoms are stored contiguously, atom by atom, in the
// batch's region of B * kRecCap records, so both the packing writes and the
// compute reads are contiguous across lanes.
template <typename real>
struct Rec;
template <>
struct alignas(16) Rec<float> {
    int jm;
    float dx, dy, dz;
};
template <>
struct alignas(16) Rec<double> {
    int jm, pad;
    double dx, dy, dz;
};

// jm: bits 0-23 index of n (at most 2^24 atoms); bits 24-25 type of n;
// bit 26: r_in < cutoff of entry (t_i, t_n, t_n) (n is a bond partner);
// bit 27 + t: r_in < cutoff of entry (t_i, t, t_n) (n is a third atom for a
// partner of type t).
constexpr int kIdMask = (1 << 24) - 1;
constexpr int kTypeShift = 24;
constexpr int kPairBit = 26;
constexpr int kThirdBit = 27;
static_assert(kMaxTypes <= 4, "two type bits and four third-atom bits per record");
__device__ __forceinline__ int rec_type(int jm) { return (jm >> kTypeShift) & 3; }

// 64-entry chunks of the packing kernel whose loads are issued together: 8,
// and 4 for the several-species float records, whose tables and types take
// registers enough that 8 would cost two wavefronts per SIMD (2M-atom
// silicon: 4 and 8 equal in mixed, FP64 252 against 227 us; 256k-atom two
// species, mixed: 40 against 44 us)
template <typename real, bool ONE>
constexpr int pack_chunks() { return (!ONE && sizeof(real) == 4) ? 4 : 8; }
constexpr int kOwnerCap = 1024;   // batch entries whose atom is looked up in a table (the rest: binary search)
static_assert(kKeptFast == 8, "the first block of a kept list is two 16-byte words");

// Position of atom `who` in the kept-neighbour list of atom m (-1: absent);
// `absent` tells that `who` is certainly not in the list (a list truncated
// at kRecCap entries, whose tail is unknown, leaves it false).  A kept list
// is in ascending order (the order of the sorted neighbour row), so the
// position is the number of entries below `who`; the -1 end markers compare
// above every index as unsigned.  Both 16-byte words of the first block are
// loaded together.
__device__ __forceinline__ int kept_position(const int *__restrict__ kept, const int *__restrict__ kept_more,
                                             int m, int who, bool &absent)
{
    const int4 *kb = reinterpret_cast<const int4 *>(kept + (size_t)m * kKeptFast);
    const int4 v0 = kb[0], v1 = kb[1];
    const unsigned w = (unsigned)who;
    const unsigned v[kKeptFast] = {(unsigned)v0.x, (unsigned)v0.y, (unsigned)v0.z, (unsigned)v0.w,
                                   (unsigned)v1.x, (unsigned)v1.y, (unsigned)v1.z, (unsigned)v1.w};
    // entries below who: the sign bit of min(v, 2^31 - 1) - who (indices < 2^24;
    // the -1 end markers clamp to 2^31 - 1, above every index); who is in the
    // list when the smallest v xor who is 0
    unsigned b[kKeptFast], x[kKeptFast];
#pragma unroll
    for (int q = 0; q < kKeptFast; ++q) {
        b[q] = (min(v[q], 0x7fffffffu) - w) >> 31;
        x[q] = v[q] ^ w;
    }
    const int pos = (int)(b[0] + b[1] + b[2] + b[3] + b[4] + b[5] + b[6] + b[7]);
    const unsigned mn = min(min(min(x[0], x[1]), min(x[2], x[3])), min(min(x[4], x[5]), min(x[6], x[7])));
    absent = false;
    if (mn == 0u) return pos;
    if (v1.w < 0 || pos < kKeptFast) {
        absent = true;   // the list ended, or passed who
        return -1;
    }
    // the list goes on past its first block and every entry so far is below who
    const int *km = kept_more + (size_t)m * kRecCap;
#pragma unroll 1
    for (int q = kKeptFast; q < kRecCap; ++q) {
        const int xx = km[q];
        if (xx == who) return q;
        if (xx < 0 || xx > who) {
            absent = true;
            return -1;
        }
    }
    return -1;
}
constexpr int kScap = 64;      // packed slots per compute batch (one per lane)
// Resident packing wavefronts per CU: more than this only adds contention for
// the CU's vector-memory path (the kernel is bound by its neighbour-position
// gathers, not by latency).
constexpr int kPackWavesPerCU = 24;
// Resident compute wavefronts per CU (the grid is persistent), by precision:
// past these the extra wavefronts cost more than they hide in latency
// (measured on the 2M-atom silicon workload, caps of 8/10/12/16 and none:
// mixed and all-FP32 fastest at 16, four per SIMD; FP64 at 10 -- 369 us
// against 465 us at 12 or more).
constexpr int kComputeWavesPerCU[kNumPrec] = {10, 16, 16};   // FP64, mixed, single

// ------------------------------------------------------------- pack kernel -
//
// Lanes = list entries of B consecutive centre atoms (their rows flattened
// through a prefix count of the row lengths).  Each lane computes the FP64 minimum-image displacement and r^2 of
// its entry and keeps it if r^2 is below the (symmetric) packing radius; the
// kept entries are written, atom by atom and in list order, to the batch's
// record region, and each atom's kept neighbours, in the same order, to its
// kept-neighbour list.  Because the radius is symmetric and r^2 of (i, n) and
// (n, i) is bit-identical, i keeps n exactly when n keeps i, so the centre i
// finds where atom n expects the force of i's terms -- force plane k, k the
// position of i in n's kept list -- by looking i up in that list.
//
// BATCHED: the atoms belong to several systems (each row holds atoms of its
// own system only); every centre atom uses its system's box, and there is no
// stale check (a batch is built and evaluated together).
template <typename real, bool ONE, bool BATCHED>
__global__ __launch_bounds__(kWave) void k_pack(PackLaunch a, DeviceTable tab)
{
    __shared__ double xi[kWave], yi[kWave], zi[kWave];
    __shared__ double bL[BATCHED ? 3 : 1][BATCHED ? kWave : 1], biL[BATCHED ? 3 : 1][BATCHED ? kWave : 1];
    __shared__ int ti[kWave], cnt[kWave], cid[kWave];   // type, kept count and atom of each batch slot
    __shared__ int eoff[kWave + 1];
    __shared__ int kst[kKeptFast][kWave];   // first kept neighbours of the batch's atoms
    __shared__ unsigned char owner[kOwnerCap];   // batch atom of each of the first kOwnerCap entries
    // radius tables, read before the first store so that no reload of them
    // has to wait behind the record stores
    __shared__ double psq_s[ONE ? 1 : kMaxTypes * kMaxTypes];
    __shared__ double cut_s[ONE ? 1 : kMaxTypes * kMaxTypes * kMaxTypes];
    constexpr int kCh = pack_chunks<real, ONE>();
    const int lane = threadIdx.x;
    Rec<real> *recs = static_cast<Rec<real> *>(a.recs);
    const int B = a.atoms_per_batch;
    const int n = BATCHED ? *a.n_dev : a.n;
    const int nbatch = (n + B - 1) / B;
    const double psq0 = tab.packsq[0];
    if constexpr (!ONE) {
        const int nt = tab.ntypes;
        for (int q = lane; q < nt * nt; q += kWave) psq_s[q] = tab.packsq[q];
        for (int q = lane; q < nt * nt * nt; q += kWave) cut_s[q] = tab.px[q].cutsq;
    }

    const ItemRange items = xcd_items(nbatch);
    // the per-atom inputs of a batch, loaded one batch ahead so that their
    // latency overlaps the previous batch
    struct AtomIn {
        double x, y, z, bx, by, bz;
        int rc, t, id;
    };
    auto fetch = [&](int b, AtomIn &v) {
        v.rc = 0;
        if (b < items.end && lane < min(B, n - b * B)) {
            const int slot = b * B + lane;
            const size_t i = (size_t)slot;
            v.id = (int)i;
            v.x = a.pos[3 * i]; v.y = a.pos[3 * i + 1]; v.z = a.pos[3 * i + 2];
            v.t = ONE ? 0 : a.types[i];
            v.rc = a.row_count[i];
            if constexpr (!BATCHED) {
                v.bx = a.pos_build[3 * i]; v.by = a.pos_build[3 * i + 1]; v.bz = a.pos_build[3 * i + 2];
            }
        }
    };
    AtomIn nxt;
    fetch(items.begin, nxt);
    for (int bt = items.begin; bt < items.end; bt += items.stride) {
        const int a0 = bt * B;
        const int nb = min(B, n - a0);
        const AtomIn cur = nxt;
        fetch(bt + items.stride, nxt);
        if (lane < nb) {
            const size_t i = (size_t)cur.id;
            xi[lane] = cur.x; yi[lane] = cur.y; zi[lane] = cur.z;
            ti[lane] = cur.t;
            cid[lane] = cur.id;
            cnt[lane] = 0;
            if constexpr (BATCHED) {
                const CellGrid &g = a.sys[a.sys_of[i]].g;
                for (int d = 0; d < 3; ++d) {
                    bL[d][lane] = g.L[d];
                    biL[d][lane] = g.invL[d];
                }
            } else {
                const double dx = cur.x - cur.bx, dy = cur.y - cur.by, dz = cur.z - cur.bz;
                if (!(dx * dx + dy * dy + dz * dz <= a.stale_sq)) atomicOr(a.flags, kFlagStale);
            }
        }
        {
            // local entry offsets of the batch's rows
            const int rc = lane < nb ? cur.rc : 0;
            const int inc = wave_incl_scan(rc);
            if (lane < nb) eoff[lane + 1] = inc;
            if (lane == 0) eoff[0] = 0;
            for (int e = inc - rc; e < min(inc, kOwnerCap); ++e) owner[e] = (unsigned char)lane;
        }
        __syncthreads();
        const int e_begin = eoff[0], e_end = eoff[nb];
        int npacked = 0;   // kept entries of the batch so far (records beyond an atom's cap excluded)
        for (int eb = e_begin; eb < e_end; eb += kWave * kCh) {
            // All loads of the kCh chunks are issued unconditionally (lanes
            // past the batch's last entry re-read that entry and are masked
            // below): a load inside a branch is waited for at the branch's end,
            // which would serialise the chunks' gathers.
            int jv[kCh], tv[kCh];
            double xv[kCh], yv[kCh], zv[kCh];
            int alv[kCh];
#pragma unroll
            for (int c = 0; c < kCh; ++c) {
                const int ec = min(eb + c * kWave + lane, e_end - 1);
                const int al = ec < kOwnerCap ? (int)owner[ec] : find_seg(eoff, nb, ec);
                alv[c] = al;
                // row-buffer index of the entry
                jv[c] = a.ell[(size_t)cid[al] * a.cap + (ec - eoff[al])];
            }
#pragma unroll
            for (int c = 0; c < kCh; ++c) {
                const double *pj = a.pos + 3 * (size_t)jv[c];
                xv[c] = pj[0]; yv[c] = pj[1]; zv[c] = pj[2];
                tv[c] = ONE ? 0 : a.types[jv[c]];
            }
#pragma unroll
            for (int c = 0; c < kCh; ++c) {
                const int e0 = eb + c * kWave;
                if (e0 >= e_end) break;
                const int e = e0 + lane;
                bool acc = false;
                int al = 0;
                double dx = 0, dy = 0, dz = 0, rsq = 0;
                if (e < e_end) {
                    al = alv[c];
                    if constexpr (BATCHED) {
                        dx = image(xv[c] - xi[al], bL[0][al], biL[0][al]);
                        dy = image(yv[c] - yi[al], bL[1][al], biL[1][al]);
                        dz = image(zv[c] - zi[al], bL[2][al], biL[2][al]);
                    } else {
                        dx = image(xv[c] - xi[al], a.L[0], a.invL[0]);
                        dy = image(yv[c] - yi[al], a.L[1], a.invL[1]);
                        dz = image(zv[c] - zi[al], a.L[2], a.invL[2]);
                    }
                    rsq = norm2(dx, dy, dz);
                    const double psq = ONE ? psq0 : psq_s[ti[al] * tab.ntypes + tv[c]];
                    acc = rsq < psq;
                }
                const unsigned long long m = __ballot(acc);
                // rank of this entry among the kept entries of its atom
                const int first = max(eoff[al] - e0, 0);
                const unsigned long long below = (lane ? (~0ull >> (64 - lane)) : 0ull);
                const unsigned long long from = first ? ~(~0ull >> (64 - first)) : ~0ull;
                const int k = cnt[al] + __popcll(m & below & from);
                const unsigned long long mrec = __ballot(acc && k < kRecCap);
                if (acc) {
                    if (k < kRecCap) {
                        if (k < kKeptFast) kst[k][al] = jv[c];
                        else a.kept_more[(size_t)cid[al] * kRecCap + k] = jv[c];
                        Rec<real> o;
                        int mask = jv[c] | (tv[c] << kTypeShift);
                        if (ONE) {
                            mask |= (1 << kPairBit) | (1 << kThirdBit);
                        } else {
                            const int nt = tab.ntypes, t_i = ti[al], t_n = tv[c];
                            if (rsq < cut_s[(t_i * nt + t_n) * nt + t_n]) mask |= 1 << kPairBit;
                            for (int t = 0; t < nt; ++t)
                                if (rsq < cut_s[(t_i * nt + t) * nt + t_n]) mask |= 1 << (kThirdBit + t);
                        }
                        o.jm = mask;
                        o.dx = (real)dx;
                        o.dy = (real)dy;
                        o.dz = (real)dz;
                        if constexpr (sizeof(real) == 8) o.pad = 0;
                        // batch order: slot = kept entries of the batch before this one
                        const size_t slot = (size_t)a0 * kRecCap + npacked + lanes_below(mrec);
                        recs[slot] = o;
                        if constexpr (sizeof(real) == 4) {
                            // rounding error of the compute kernel's FP32 distance
                            // (the same operations on the same float displacement)
                            // (rsq - rf^2 is exact: rf^2 has 48 bits and the two
                            // agree to ~1e-7, Sterbenz; r - rf = (rsq - rf^2) / (2 rf)
                            // up to a relative 5e-8 of itself)
                            const float rf = __builtin_amdgcn_sqrtf(norm2r(o.dx, o.dy, o.dz));
                            const double rfd = (double)rf;
                            a.rlo[slot] = (float)fma(-rfd, rfd, rsq) * (0.5f * __builtin_amdgcn_rcpf(rf));
                        }
                    }
                }
                npacked += __popcll(mrec);
                __syncthreads();
                if (acc) atomicMax(&cnt[al], k + 1);
                __syncthreads();
            }
        }
        if (lane < nb) {
            const int i = cur.id;
            int c = cnt[lane];
            // the kept list: its first block, and the end marker
            int4 *kb = reinterpret_cast<int4 *>(a.kept + (size_t)i * kKeptFast);
            int kv[kKeptFast];
#pragma unroll
            for (int q = 0; q < kKeptFast; ++q) kv[q] = q < c ? kst[q][lane] : -1;
            kb[0] = make_int4(kv[0], kv[1], kv[2], kv[3]);
            kb[1] = make_int4(kv[4], kv[5], kv[6], kv[7]);
            if (c >= kKeptFast && c < kRecCap) a.kept_more[(size_t)i * kRecCap + c] = -1;
            if (c > kRecCap) {
                // more kept neighbours than its records hold: the atom is
                // evaluated with its first kRecCap neighbours only and the
                // result is reported invalid; k_fixup_dropped zeroes the force
                // slots its neighbours reserved for it
                atomicOr(a.flags, kFlagOverflow);
                a.drop_list[atomicAdd(a.drop_count, 1)] = i;
                c = kRecCap;
            }
            a.pcount[i] = c;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------- compute kernel -

// Three-body parameters of one table entry (the quantities of g(theta) and of
// the exponential factor of Eq. 3), staged in LDS by the kernels for several
// species.
template <typename real>
struct TripParam {
    real h, gamma, c2d2, d2, two_c2, lam3, lam3m, m;
};

template <typename real>
__device__ __forceinline__ TripParam<real> trip_of(const ParamR<real> &p)
{
    return {p.h, p.gamma, p.c2d2, p.d2, p.two_c2, p.lam3, p.lam3m, p.m};
}

template <typename real, int NT>
struct Shared {
    // per centre atom of the batch
    int ti[kWave];
    int cid[kWave];              // its atom index
    int pcnt[kWave];
    int pstart[kWave + 1];
    unsigned char owner[kScap];  // centre atom (batch index) of each slot
    // per packed slot (i, n)
    double fs[kScap][3];         // force on n from i's terms (FP64)
    real ux[kScap], uy[kScap], uz[kScap], r[kScap];
    real dzeta[kScap];           // dV(i,n,zeta_in)/dzeta
    int mask[kScap];
    real fc[NT][kScap], dfc[NT][kScap];   // f_C(r_in), f_C'(r_in) of entry (t_i, t, t_n), per partner type t
    real ep[kScap], em[kScap];            // exp(lambda3 r_in), exp(-lambda3 r_in) (one type, m = 1)
};

// Records of the fused packing: a ring of kQueueCap records (with their
// FP32 distance corrections and force-plane indices) and the row layout of
// the group's centre atoms.
constexpr int kQueueCap = kScap + kScap + kRecCap;

template <typename real>
struct FusedQueue {
    Rec<real> rec[kQueueCap];
    float rlo[kQueueCap];
    unsigned char rev[kQueueCap];   // position of the centre in the neighbour's row
    int cnt[kWave];                 // kept entries so far of each atom of the group
    int eoff[kWave + 1];            // first entry of each atom's row (group-local)
    int ti[kWave];
};

// The k-role quantities of triplet (i; k, j) -- pair (i, k) with j as its
// third atom -- that the first K loop of lane (i, j) forms alongside its own
// triplet (i; j, k) (same angle, same g and g' when the three-body parameters
// are symmetric in j and k): v = g' e (u_k - cos u_j), s = g e, with e the
// exponential factor of pair (i, k) and third atom j.
template <typename real>
struct alignas(4 * sizeof(real)) KCache {
    real vx, vy, vz, s;
};

template <typename real>
struct Angular {
    real g, dg;   // g(theta) and dg/dcos(theta)
};

// g(theta) = gamma (1 + c^2/d^2 - c^2/(d^2 + (cos - h)^2)) written without
// cancellation as gamma + (gamma c^2/d^2) t^2 / (d^2 + t^2), t = cos - h, and
// g' = 2 gamma c^2 t / (d^2 + t^2)^2.
template <typename real, typename Q>
__device__ __forceinline__ Angular<real> angular(const Q &q, real cs)
{
    const real t = cs - q.h;
    const real iden = M<real>::rcp(q.d2 + t * t);
    Angular<real> a;
    a.g = q.gamma + q.c2d2 * (t * t) * iden;      // c2d2 = gamma c^2 / d^2
    a.dg = q.two_c2 * t * (iden * iden);           // two_c2 = 2 gamma c^2
    return a;
}

// exp((lambda3 (rj - rk))^m) and its derivative with respect to rj.
template <typename real, typename Q>
__device__ __forceinline__ void exp_term(const Q &q, real rj, real rk, real &ex, real &dex)
{
    ex = real(1);
    dex = real(0);
    if (q.lam3 != real(0)) {
        const real dr = rj - rk;
        if (q.m == real(3)) {
            const real dr2 = dr * dr;
            ex = M<real>::exp(q.lam3m * dr2 * dr);
            dex = real(3) * q.lam3m * dr2 * ex;
        } else {
            ex = M<real>::exp(q.lam3 * dr);
            dex = q.lam3 * ex;
        }
    }
}

// (d/d rj) exp((lambda3 (rj - rk))^m) / exp((lambda3 (rj - rk))^m).
template <typename real, typename Q>
__device__ __forceinline__ real exp_ratio(const Q &q, real rj, real rk)
{
    if (q.lam3 == real(0)) return real(0);
    if (q.m == real(3)) {
        const real dr = rj - rk;
        return real(3) * q.lam3m * dr * dr;
    }
    return q.lam3;
}

// Eq. (2) of pair (i, j) once zeta_ij is known: the pair's energy (half of
// f_C (f_R + b f_A); each bond is visited from both ends), dV/dzeta_ij, and
// the pair force on j (along u_ij), in FP64, or in FP32 in the single variant.
template <typename real, bool SINGLE, typename facc>
__device__ __forceinline__ void pair_step(const ParamR<real> &q, const ParamX &px, real zr, real fc, real dfc,
                                          real rj, real rjlo, const real uj[3], double &e_pair, real &dz_out,
                                          facc &fx, facc &fy, facc &fz)
{
    // Eq. (2) in log form: FP64, or FP32 in the single variant
    if constexpr (sizeof(real) == 4 && !SINGLE) {
        // mixed: f_R and f_A from the FP32 pair exponential of
        // the FP64 distance, combined in FP64 (at short range
        // f_R' and b f_A' cancel to a few percent of either)
        const double fr = exp_decay_f32(px.A, q.lam1, q.lam1_lo, rj, rjlo);
        const double fa = -exp_decay_f32(px.B, q.lam2, q.lam2_lo, rj, rjlo);
        const double zeta = (double)zr;
        double b = 1.0, db = 0.0;
        if (zeta > 0.0) bond_order_f64(px, zeta, b, db);
        const double fc64 = (double)fc, vp = fr + b * fa;
        e_pair = 0.5 * fc64 * vp;
        dz_out = (real)(0.5 * fc64 * fa * db);
        const double dvdr = 0.5 * ((double)dfc * vp - fc64 * (px.lam1 * fr + b * (px.lam2 * fa)));
        fx = -dvdr * (double)uj[0];
        fy = -dvdr * (double)uj[1];
        fz = -dvdr * (double)uj[2];
    } else if constexpr (SINGLE) {
        real fr, fa, dfr, dfa;
        pair_terms(q, rj, fr, dfr, fa, dfa, rjlo);
        // b - 1 is carried instead of b (b is within ~1e-4 of 1,
        // and its FP32 rounding would bias the energy through
        // the large f_A at short range); ln(beta zeta) is taken
        // of the product (ln beta ~ -14 and ln zeta ~ 10 would
        // each carry a float rounding ~1e-6 into the sum)
        float bm1 = 0.f, db = 0.f;
        if (zr > 0.f) {
            const float x = expf((float)px.eta * logf(q.beta * zr));
            bm1 = expm1f(-log1pf(x) * (float)px.inv2eta);
            db = -0.5f * (1.f + bm1) * x / (zr * (1.f + x));
        }
        e_pair = (double)(0.5f * fc * ((fr + fa) + bm1 * fa));
        dz_out = 0.5f * fc * fa * db;
        const real dvdr1 = real(0.5) * (dfc * ((fr + fa) + bm1 * fa) + fc * ((dfr + dfa) + bm1 * dfa));
        fx = -dvdr1 * uj[0];
        fy = -dvdr1 * uj[1];
        fz = -dvdr1 * uj[2];
    } else {
        // all-FP64 path, with the library's exp / log / log1p
        real fr, fa, dfr, dfa;
        pair_terms(q, rj, fr, dfr, fa, dfa);
        const double zeta = (double)zr;
        double b = 1.0, db = 0.0;
        if (zeta > 0.0) {
            const double x = ::exp(px.eta * (px.logbeta + ::log(zeta)));
            b = ::exp(-::log1p(x) * px.inv2eta);
            db = -0.5 * b * x / (zeta * (1.0 + x));
        }
        e_pair = 0.5 * fc * (fr + b * fa);
        dz_out = 0.5 * fc * fa * db;
        const real dvdr = real(0.5) * (dfc * (fr + b * fa) + fc * (dfr + b * dfa));
        fx = -dvdr * uj[0];
        fy = -dvdr * uj[1];
        fz = -dvdr * uj[2];
    }
}

// The workgroup's partial sums of energy and virial, its pair and triplet
// counts and its asymmetry flag, summed across the wavefront and stored by
// lane 0 at the workgroup's index (reduced by the gather kernel).
__device__ __forceinline__ void store_partials(const ComputeLaunch &a, double e_acc, const double w_acc[6],
                                               int n_pairs, int n_trip, bool asym)
{
    double v[7] = {e_acc, w_acc[0], w_acc[1], w_acc[2], w_acc[3], w_acc[4], w_acc[5]};
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = wave_sum(v[c]);
    long long np = n_pairs, ntr = n_trip;   // summed across the wavefront in 64 bits
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        np += __shfl_xor(np, off, kWave);
        ntr += __shfl_xor(ntr, off, kWave);
    }
    const bool any_asym = __ballot(asym) != 0ull;
    if (threadIdx.x == 0) {
        double *pp = a.partials + 8 * (size_t)blockIdx.x;
        pp[7] = any_asym ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < 7; ++c) pp[c] = v[c];
        a.counters[2 * (size_t)blockIdx.x] = np;
        a.counters[2 * (size_t)blockIdx.x + 1] = ntr;
    }
}

// One 64-lane wavefront per workgroup walks batches of consecutive centre
// atoms whose packed neighbours fill at most one slot per lane; a lane owns
// the pair (i, j) of its slot (the pair-vectorised scheme of Section 3 with
// pairs of several centre atoms side by side):
//   1  first K loop over the other slots k of centre i: zeta_ij, and with the
//      same cos(theta_ijk), g and g' the derivative dzeta_ij/dx_j (Section 2:
//      zeta and its derivatives formed once); CACHE also keeps, per k, the
//      k-role quantities of triplet (i; k, j) in LDS;
//   2  f_C, f_R, f_A, b_ij and db/dzeta in FP64 log form, energy, pair force,
//      dV/dzeta_ij (shared through LDS); the j-role force
//      -dV/dzeta_ij dzeta_ij/dx_j follows at once;
//   3  second K loop: the k-role terms -dV/dzeta_ik dzeta(i,k,j)/dx_j, each
//      a product of dV/dzeta_ik with the cached quantities (recomputed past
//      the cache, or when the parameters are not symmetric in j and k); the
//      lane sums every force term of centre i on atom j in FP64, so no two
//      lanes ever update the same force;
//   4  virial d_ij (x) F_j; the force on i is minus the sum over its slots.
// Each slot's force goes to the slot atom j reserved for centre i (plane k
// of the per-atom force planes, k the position of i in j's kept list), each
// centre's own force to `own`; k_gather_forces sums them per atom.
//
// NT: 1 (one species: the single entry in registers), 2 or kMaxTypes (the
// three-body part of the table staged in LDS).  CACHE: the three-body
// parameters of (ti, tj, tk) and (ti, tk, tj) agree (always for one species).
//
// BATCHED: the batch holds several systems; each centre atom's energy and
// virial (the sums over its slots) are stored per atom for the per-system
// reduction, in place of the per-workgroup partial sums.
//
// SINGLE (with real = float): the all-FP32 variant -- the zeta -> b power and
// each lane's sum of the force terms on j in FP32 as well; FP64 remains only
// in the displacement (packing) and in the sums across lanes and atoms.
template <typename real, int NT, bool BATCHED, bool SINGLE, bool NOL3, bool CACHE, bool ATOMIC = false,
          bool FUSED = false>
__global__ __launch_bounds__(kWave) void k_tersoff(ComputeLaunch a, DeviceTable tab)
{
    static_assert(!(ATOMIC && BATCHED), "the atomic scatter serves one system");
    static_assert(!SINGLE || sizeof(real) == 4, "the single-precision variant computes in float");
    static_assert(!NOL3 || NT == 1, "the lambda3-free variant is a one-species kernel");
    constexpr bool ONE = NT == 1;
    using facc = typename std::conditional<SINGLE, float, double>::type;   // per-lane force sum
    // float paths: the FP64 distance enters the pair terms as r + r_lo
    constexpr bool kRlo = sizeof(real) == 4;
    constexpr int KC = CACHE ? (sizeof(real) == 4 ? 4 : 3) : 1;   // cached k per lane
    constexpr int kPlaneCap = FUSED ? kFusedRowCap : kRecCap;   // force planes per atom
    __shared__ Shared<real, NT> sh;
    __shared__ KCache<real> kc[KC][kScap];
    __shared__ TripParam<real> tp[ONE ? 1 : NT * NT * NT];
    __shared__ double sev[BATCHED ? kScap : 1][BATCHED ? 7 : 1];   // per-slot energy and virial
    const int lane = threadIdx.x;
    const ParamR<real> *ptab = table_r<real>(tab);
    const Rec<real> *recs = static_cast<const Rec<real> *>(a.recs);
    const int nt = ONE ? 1 : tab.ntypes;
    if constexpr (!ONE) {
        for (int e = lane; e < nt * nt * nt; e += kWave) tp[e] = trip_of(ptab[e]);
    }
    // one species: the single entry, held in registers; the m = 1 factor
    // exp(lambda3 (r_ij - r_ik)) then separates into per-slot exponentials
    // (when they stay far from overflow)
    const ParamR<real> q0 = ptab[0];
    const TripParam<real> t0 = trip_of(q0);
    const bool sep = !NOL3 && ONE && q0.m == real(1) && q0.lam3 != real(0) &&
                     fabs((double)q0.lam3) * (double)q0.Rc < 40.0;
    auto trip = [&](int e) -> TripParam<real> {
        if constexpr (ONE) return t0;
        else return tp[e];
    };

    double e_acc = 0.0;
    double w_acc[6] = {0, 0, 0, 0, 0, 0};
    int n_pairs = 0, n_trip = 0;   // this lane's (well below 2^31 per lane)
    bool asym = false;   // a kept neighbour whose (complete) kept list lacks the centre

    const int B = a.atoms_per_batch;
    const int n = BATCHED ? *a.n_dev : a.n;
    const int ngroups = (n + B - 1) / B;

    const ItemRange items = xcd_items(ngroups);
    // The inputs of a batch are loaded one batch ahead, while the previous
    // batch computes: its atoms' record counts and types, and the first kScap
    // records of its place in the group's region (its own slots: records are
    // stored in batch order).  A group of B atoms owns B * kRecCap records;
    // loads never pass its end.
    struct Ahead {
        int grp, a0, a_end;   // group, first atom, end of the group's atoms
        size_t rec;           // index of the batch's first record
        int p, t, id;         // this lane's atom: record count, type, index
        Rec<real> rc;         // this lane's slot record
        float rlo;
    };
    auto fetch = [&](Ahead &f) {
        f.p = 0;
        f.t = 0;
        f.id = 0;
        if (lane < f.a_end - f.a0) {
            const int slot = f.a0 + lane;
            f.id = slot;
            f.p = a.pcount[f.id];
            f.t = ONE ? 0 : a.types[f.id];
        }
        if (f.rec + lane < (size_t)(f.grp + 1) * B * kRecCap) {
            f.rc = recs[f.rec + lane];
            if constexpr (kRlo) f.rlo = a.rlo[f.rec + lane];
        }
    };
    auto group_start = [&](Ahead &f, int g) {
        f.grp = g;
        f.a0 = g * B;
        f.a_end = min(f.a0 + B, n);
        f.rec = (size_t)f.a0 * kRecCap;
    };
    // One batch: the leading atoms from batch slot a0 (nb available) whose
    // slots fit one per lane.  Lane inputs: p, tiv, cid_in -- the slot count,
    // type and index of the atom at batch slot a0 + lane; rc_ahead, rlo_ahead
    // -- the record of slot lane; kpos_in -- (fused packing) the force plane
    // of the slot.  after_header(cut, npacked) runs once the batch is formed,
    // after_slots() once the slot inputs are consumed.  Returns (atoms,
    // slots) of the batch.
    auto run_batch = [&](const int a0, const int nb, const int p, const int tiv, const int cid_in,
                         const Rec<real> rc_ahead, const float rlo_ahead, const int kpos_in, auto &&after_header,
                         auto &&after_slots) -> int2 {
        // ---- batch: the leading atoms whose slots fit one per lane
        const int ip = wave_incl_scan(p);
        const int cut = __popcll(__ballot(lane < nb && ip <= kScap));   // >= 1: p <= kRecCap
        if (lane < cut) {
            sh.ti[lane] = tiv;
            sh.cid[lane] = cid_in;
            sh.pcnt[lane] = p;
            sh.pstart[lane + 1] = ip;
            for (int q = ip - p; q < ip; ++q) sh.owner[q] = (unsigned char)lane;
        }
        if (lane == 0) sh.pstart[0] = 0;
        const int npacked = __shfl(ip, cut - 1, kWave);
        __syncthreads();
        after_header(cut, npacked);

        // ---- slot lanes: load the packed record of pair (i, j), and the
        // switching function of the slot for every partner type
        const int s = lane;
        const bool has_slot = s < npacked;
        int al = 0, jl = 0, pc = 0, sb = 0, j = 0, kpos = -1, mj = 0, ti = 0;
        real rj = 0, rjinv = 0, rjlo = 0, uj[3] = {0, 0, 0}, dj[3] = {0, 0, 0};
        if (has_slot) {
            al = sh.owner[s];
            sb = sh.pstart[al];
            jl = s - sb;
            pc = sh.pcnt[al];
            ti = ONE ? 0 : sh.ti[al];
            const Rec<real> rc = rc_ahead;
            if constexpr (kRlo) rjlo = rlo_ahead;
            j = rc.jm & kIdMask;
            if constexpr (FUSED) {
                kpos = kpos_in;
            } else if constexpr (!ATOMIC) {
                bool absent;
                kpos = kept_position(a.kept, a.kept + (size_t)kKeptFast * a.plane_stride, j, sh.cid[al], absent);
                asym |= absent;
            }
            mj = rc.jm;
            dj[0] = rc.dx; dj[1] = rc.dy; dj[2] = rc.dz;
            rj = M<real>::sqrt(norm2r(dj[0], dj[1], dj[2]));
            rjinv = M<real>::rcp(rj);
            uj[0] = dj[0] * rjinv; uj[1] = dj[1] * rjinv; uj[2] = dj[2] * rjinv;
            sh.ux[s] = uj[0]; sh.uy[s] = uj[1]; sh.uz[s] = uj[2];
            sh.r[s] = rj;
            sh.mask[s] = mj;
            for (int t = 0; t < nt; ++t) {
                real fc = real(0), dfc = real(0);
                if ((mj >> (kThirdBit + t)) & 1)
                    cutoff_terms(ONE ? q0 : ptab[(ti * nt + t) * nt + rec_type(mj)], rj, fc, dfc, rjlo);
                sh.fc[t][s] = fc;
                sh.dfc[t][s] = dfc;
            }
            if (sep) {
                sh.ep[s] = M<real>::exp(q0.lam3 * rj);
                sh.em[s] = M<real>::exp(-q0.lam3 * rj);
            }
        }
        after_slots();   // this batch's inputs are consumed
        __syncthreads();

        // exp((lambda3 (r_a - r_b))^m) and its derivative with respect to r_a
        auto ex_term = [&](const TripParam<real> &q, int sa, real ra, int sbb, real rbb, real &ex, real &dex) {
            if constexpr (NOL3) {
                ex = real(1);   // lambda3 = 0: the factor is 1 in every triplet
                dex = real(0);
            } else if (ONE && sep) {
                ex = sh.ep[sa] * sh.em[sbb];
                dex = q0.lam3 * ex;
            } else {
                exp_term(q, ra, rbb, ex, dex);
            }
        };

        const int tj = rec_type(mj);
        const bool j_pair = ONE || ((mj >> kPairBit) & 1);
        facc fx = 0, fy = 0, fz = 0;       // force on j from centre i's terms
        double e_pair = 0.0;   // energy of pair (i, j)
        if (has_slot) {
            // ---- 1: zeta_ij and dzeta_ij/dx_j = aj / r_ij + bj u_ij over the
            // other slots k of centre i (k = j skipped by the index map)
            real zr = real(0), aj[3] = {0, 0, 0}, bj = real(0);
            if (CACHE || j_pair) {
                for (int kk = 0; kk + 1 < pc; ++kk) {
                    const int sk = sb + kk + (kk >= jl ? 1 : 0);
                    const int mk = ONE ? 0 : sh.mask[sk];
                    const int tk = ONE ? 0 : rec_type(mk);
                    const TripParam<real> q = trip((ti * nt + tj) * nt + tk);
                    const real rk = sh.r[sk];
                    const real uk[3] = {sh.ux[sk], sh.uy[sk], sh.uz[sk]};
                    const real cs = uj[0] * uk[0] + uj[1] * uk[1] + uj[2] * uk[2];
                    const Angular<real> an = angular(q, cs);
                    // r_ij d cos(theta_ijk) / d x_j
                    const real tv[3] = {uk[0] - cs * uj[0], uk[1] - cs * uj[1], uk[2] - cs * uj[2]};
                    real ex, dex;
                    ex_term(q, s, rj, sk, rk, ex, dex);
                    const bool member = j_pair && (ONE || ((mk >> (kThirdBit + tj)) & 1));
                    const real fck = member ? sh.fc[ONE ? 0 : tj][sk] : real(0);
                    const real fg = fck * an.g;
                    zr += fg * ex;
                    const real w = fck * an.dg * ex;
                    aj[0] += w * tv[0];
                    aj[1] += w * tv[1];
                    aj[2] += w * tv[2];
                    bj += fg * dex;
                    if constexpr (!ONE) n_trip += member ? 1 : 0;
                    if constexpr (CACHE) {
                        if (kk < KC) {
                            real ex2, dex2;
                            ex_term(q, sk, rk, s, rj, ex2, dex2);
                            const real w2 = an.dg * ex2;
                            kc[kk][s] = KCache<real>{w2 * tv[0], w2 * tv[1], w2 * tv[2], an.g * ex2};
                        }
                    }
                }
            }
            // ---- 2: pair terms, bond order, dV/dzeta
            real dz_out = real(0);
            if (j_pair) {
                ++n_pairs;
                if constexpr (ONE) n_trip += pc - 1;   // every other slot is a third atom
                const int e_ij = ONE ? 0 : (ti * nt + tj) * nt + tj;
                const ParamR<real> &q = ONE ? q0 : ptab[e_ij];
                const ParamX px = tab.px[e_ij];
                const real fc = sh.fc[ONE ? 0 : tj][s], dfc = sh.dfc[ONE ? 0 : tj][s];
                pair_step<real, SINGLE>(q, px, zr, fc, dfc, rj, rjlo, uj, e_pair, dz_out, fx, fy, fz);
                e_acc += e_pair;
                // j-role terms: -dV/dzeta_ij dzeta_ij/dx_j
                fx -= (facc)(dz_out * (aj[0] * rjinv + bj * uj[0]));
                fy -= (facc)(dz_out * (aj[1] * rjinv + bj * uj[1]));
                fz -= (facc)(dz_out * (aj[2] * rjinv + bj * uj[2]));
            }
            sh.dzeta[s] = dz_out;
        }
        __syncthreads();

        if (has_slot) {
            // ---- 3: second K loop, the k-role terms of centre i on atom j:
            // -dV/dzeta_ik dzeta(i,k,j)/dx_j over the bond partners k of i
            // that have j as a third atom, summed in the working precision
            // (a handful of triplet terms; the pair's total is stored in
            // the working precision as well)
            real ax = 0, ay = 0, az = 0, su = 0;
            for (int kk = 0; kk + 1 < pc; ++kk) {
                const int sk = sb + kk + (kk >= jl ? 1 : 0);
                const real dzk = sh.dzeta[sk];
                const int mk = ONE ? 0 : sh.mask[sk];
                const int tk = ONE ? 0 : rec_type(mk);
                const bool valid = dzk != real(0) && (ONE || ((mj >> (kThirdBit + tk)) & 1));
                const int e_kj = (ti * nt + tk) * nt + tj;
                const real rk = sh.r[sk];
                real v[3], sg, tg;   // dzeta(i,k,j)/dx_j = (fc_j v / r_j) + (fc'_j sg - fc_j tg) u_j
                if (CACHE && kk < KC) {
                    const KCache<real> c = kc[kk][s];
                    v[0] = c.vx; v[1] = c.vy; v[2] = c.vz;
                    sg = c.s;
                    if constexpr (NOL3) tg = real(0);
                    else tg = sep ? q0.lam3 * sg : sg * exp_ratio(trip(e_kj), rk, rj);
                } else {
                    const TripParam<real> q = trip(e_kj);
                    const real uk[3] = {sh.ux[sk], sh.uy[sk], sh.uz[sk]};
                    const real cs = uj[0] * uk[0] + uj[1] * uk[1] + uj[2] * uk[2];
                    const Angular<real> an = angular(q, cs);
                    real ex2, dex2;
                    ex_term(q, sk, rk, s, rj, ex2, dex2);
                    const real w2 = an.dg * ex2;
                    v[0] = w2 * (uk[0] - cs * uj[0]);
                    v[1] = w2 * (uk[1] - cs * uj[1]);
                    v[2] = w2 * (uk[2] - cs * uj[2]);
                    sg = an.g * ex2;
                    tg = an.g * dex2;
                }
                const real fcj = valid ? sh.fc[ONE ? 0 : tk][s] : real(0);
                const real dfcj = valid ? sh.dfc[ONE ? 0 : tk][s] : real(0);
                const real wv = dzk * fcj * rjinv;
                ax += wv * v[0];
                ay += wv * v[1];
                az += wv * v[2];
                su += dzk * (dfcj * sg - fcj * tg);
            }
            fx -= (facc)(ax + su * uj[0]);
            fy -= (facc)(ay + su * uj[1]);
            fz -= (facc)(az + su * uj[2]);
            // ---- 4: virial and output (FP64 from here on)
            const double Fx = (double)fx, Fy = (double)fy, Fz = (double)fz;
            const double dxj = (double)dj[0], dyj = (double)dj[1], dzj_ = (double)dj[2];
            w_acc[0] += dxj * Fx;
            w_acc[1] += dyj * Fy;
            w_acc[2] += dzj_ * Fz;
            w_acc[3] += dxj * Fy;
            w_acc[4] += dxj * Fz;
            w_acc[5] += dyj * Fz;
            if constexpr (ATOMIC) {
                double *f = a.forces_atomic + 3 * (size_t)j;
                atomicAdd(f, Fx);
                atomicAdd(f + 1, Fy);
                atomicAdd(f + 2, Fz);
            } else if ((unsigned)kpos < (unsigned)kPlaneCap) {
                real *f = static_cast<real *>(a.planes) + 3 * ((size_t)kpos * a.plane_stride + (size_t)j);
                f[0] = (real)Fx; f[1] = (real)Fy; f[2] = (real)Fz;
            }
            sh.fs[s][0] = Fx; sh.fs[s][1] = Fy; sh.fs[s][2] = Fz;
            if constexpr (BATCHED) {
                sev[s][0] = e_pair;
                sev[s][1] = dxj * Fx;
                sev[s][2] = dyj * Fy;
                sev[s][3] = dzj_ * Fz;
                sev[s][4] = dxj * Fy;
                sev[s][5] = dxj * Fz;
                sev[s][6] = dyj * Fz;
            }
        }
        __syncthreads();
        if (lane < cut) {
            double ox = 0, oy = 0, oz = 0;
            const int s0 = sh.pstart[lane], s1 = sh.pstart[lane + 1];
            for (int q = s0; q < s1; ++q) {
                ox -= sh.fs[q][0]; oy -= sh.fs[q][1]; oz -= sh.fs[q][2];
            }
            if constexpr (ATOMIC) {
                double *o = a.forces_atomic + 3 * (size_t)cid_in;
                atomicAdd(o, ox);
                atomicAdd(o + 1, oy);
                atomicAdd(o + 2, oz);
            } else {
                double *o = a.own + 3 * (size_t)cid_in;
                o[0] = ox; o[1] = oy; o[2] = oz;
            }
            if constexpr (BATCHED) {
                double v[7] = {0, 0, 0, 0, 0, 0, 0};
                for (int q = s0; q < s1; ++q)
                    #pragma unroll
                    for (int c = 0; c < 7; ++c) v[c] += sev[q][c];
                double *ea = a.eatom + 8 * (size_t)(a0 + lane);
                #pragma unroll
                for (int c = 0; c < 7; ++c) ea[c] = v[c];
                ea[7] = 0.0;
            }
        }
        __syncthreads();
        return make_int2(cut, npacked);
    };

    if constexpr (!FUSED) {
        Ahead nx{};
        nx.grp = items.end;   // an empty range (more XCD slices than groups) runs no batch
        if (items.begin < items.end) {
            group_start(nx, items.begin);
            fetch(nx);
        }
        while (nx.grp < items.end) {
            const int a0 = nx.a0, a_end = nx.a_end;
            const size_t rec0 = nx.rec;
            run_batch(a0, a_end - a0, nx.p, nx.t, nx.id, nx.rc, nx.rlo, -1,
                      [&](int cut, int npacked) {
                          // the next batch: the rest of this group, or the next group
                          nx.a0 = a0 + cut;
                          nx.rec = rec0 + npacked;
                          if (nx.a0 >= a_end) group_start(nx, nx.grp + items.stride);
                      },
                      [&]() {
                          if (nx.grp < items.end) fetch(nx);
                      });
        }
    } else {
        // ---- fused packing: each group's rows are packed here, chunk by chunk
        // of 64 entries, into a queue of records in LDS; batches are taken
        // from its head once it holds a full batch of complete atoms (or the
        // group's rows are done).  Before a chunk the queue holds fewer than
        // kScap records of complete atoms plus at most kRecCap of the one
        // atom in progress, so a chunk never overruns it.
        __shared__ FusedQueue<real> fq;
        __shared__ double psq_s[ONE ? 1 : kMaxTypes * kMaxTypes];
        __shared__ double cut_s[ONE ? 1 : kMaxTypes * kMaxTypes * kMaxTypes];
        const double psq0 = tab.packsq[0];
        if constexpr (!ONE) {
            for (int q = lane; q < nt * nt; q += kWave) psq_s[q] = tab.packsq[q];
            for (int q = lane; q < nt * nt * nt; q += kWave) cut_s[q] = tab.px[q].cutsq;
        }
        const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
        for (int grp = items.begin; grp < items.end; grp += items.stride) {
            const int g0 = grp * B, gn = min(B, n - g0);
            int rcount = 0;
            if (lane < gn) {
                const size_t i = (size_t)(g0 + lane);
                rcount = a.row_count[i];
                const double dx = a.pos[3 * i] - a.pos_build[3 * i];
                const double dy = a.pos[3 * i + 1] - a.pos_build[3 * i + 1];
                const double dz = a.pos[3 * i + 2] - a.pos_build[3 * i + 2];
                if (!(dx * dx + dy * dy + dz * dz <= a.stale_sq)) atomicOr(a.flags, kFlagStale);
                fq.ti[lane] = ONE ? 0 : a.types[i];
                fq.cnt[lane] = 0;
            }
            const int inc = wave_incl_scan(rcount);
            if (lane < gn) fq.eoff[lane + 1] = inc;
            if (lane == 0) fq.eoff[0] = 0;
            const int E = __shfl(inc, gn - 1, kWave);
            unsigned long long kb = 0;   // kept row positions of atom g0 + lane
            int e_next = 0, a_q = 0, q_head = 0, q_len = 0;
            __syncthreads();
            while (a_q < gn) {
                int a_done;
                for (;;) {
                    // atoms whose rows are done, and their records not yet computed
                    a_done = __popcll(__ballot(lane < gn && fq.eoff[lane + 1] <= e_next));
                    const int ready = wave_sum_int((lane >= a_q && lane < a_done) ? min(fq.cnt[lane], kRecCap) : 0);
                    if (ready >= kScap || e_next >= E) break;
                    const int e = e_next + lane;
                    bool acc = false;
                    int al = 0, jn = 0, rev = 0, tn = 0;
                    double dx = 0, dy = 0, dz = 0, rsq = 0;
                    if (e < E) {
                        al = find_seg(fq.eoff, gn, e);
                        const size_t q = (size_t)(g0 + al) * a.cap + (e - fq.eoff[al]);
                        jn = a.rows[q];
                        rev = a.rev[q];
                        const size_t ic = (size_t)(g0 + al);
                        dx = image(a.pos[3 * (size_t)jn] - a.pos[3 * ic], a.L[0], a.invL[0]);
                        dy = image(a.pos[3 * (size_t)jn + 1] - a.pos[3 * ic + 1], a.L[1], a.invL[1]);
                        dz = image(a.pos[3 * (size_t)jn + 2] - a.pos[3 * ic + 2], a.L[2], a.invL[2]);
                        rsq = norm2(dx, dy, dz);
                        if constexpr (!ONE) tn = a.types[jn];
                        acc = rsq < (ONE ? psq0 : psq_s[fq.ti[al] * nt + tn]);
                    }
                    const unsigned long long m = __ballot(acc);
                    // rank of this entry among the kept entries of its atom
                    const int first = max(fq.eoff[al] - e_next, 0);
                    const unsigned long long from = first ? ~(~0ull >> (64 - first)) : ~0ull;
                    const int k = fq.cnt[al] + __popcll(m & below & from);
                    const unsigned long long mrec = __ballot(acc && k < kRecCap);
                    if (acc) {
                        // rev: the position of the centre in jn's row
                        if (k < kRecCap) {
                            Rec<real> o;
                            int mask = jn | (tn << kTypeShift);
                            if (ONE) {
                                mask |= (1 << kPairBit) | (1 << kThirdBit);
                            } else {
                                const int ti_ = fq.ti[al];
                                if (rsq < cut_s[(ti_ * nt + tn) * nt + tn]) mask |= 1 << kPairBit;
                                for (int t = 0; t < nt; ++t)
                                    if (rsq < cut_s[(ti_ * nt + t) * nt + tn]) mask |= 1 << (kThirdBit + t);
                            }
                            o.jm = mask;
                            o.dx = (real)dx;
                            o.dy = (real)dy;
                            o.dz = (real)dz;
                            if constexpr (sizeof(real) == 8) o.pad = 0;
                            int qp = q_head + q_len + lanes_below(mrec);
                            if (qp >= kQueueCap) qp -= kQueueCap;
                            fq.rec[qp] = o;
                            fq.rev[qp] = (unsigned char)rev;
                            if constexpr (kRlo) {
                                // the FP64 distance minus the FP32 one the slot lane forms
                                const float rf = __builtin_amdgcn_sqrtf(norm2r(o.dx, o.dy, o.dz));
                                const double rfd = (double)rf;
                                fq.rlo[qp] = (float)fma(-rfd, rfd, rsq) * (0.5f * __builtin_amdgcn_rcpf(rf));
                            }
                        } else {
                            // beyond the atom's slots: evaluated without this
                            // neighbour and reported; the neighbour reads a zero
                            // force from this centre
                            real *f = static_cast<real *>(a.planes) + 3 * ((size_t)rev * a.plane_stride + (size_t)jn);
                            f[0] = real(0); f[1] = real(0); f[2] = real(0);
                            atomicOr(a.flags, kFlagOverflow);
                        }
                    }
                    q_len += __popcll(mrec);
                    // the chunk's kept entries into the row masks of their atoms
                    if (lane < gn) {
                        const int lo = max(fq.eoff[lane], e_next), hi = min(fq.eoff[lane + 1], e_next + kWave);
                        if (lo < hi) {
                            const int len = hi - lo;
                            const unsigned long long bits =
                                (m >> (lo - e_next)) & (len == kWave ? ~0ull : ((1ull << len) - 1ull));
                            kb |= bits << (lo - fq.eoff[lane]);
                        }
                    }
                    __syncthreads();
                    if (acc) atomicMax(&fq.cnt[al], k + 1);
                    e_next += kWave;
                    __syncthreads();
                }
                // ---- a batch from the head of the queue
                const int na = a_done - a_q;
                int p = 0, tiv = 0;
                if (lane < na) {
                    p = min(fq.cnt[a_q + lane], kRecCap);
                    tiv = fq.ti[a_q + lane];
                }
                Rec<real> rc{};
                float rl = 0.f;
                int kp = -1;
                if (lane < q_len) {
                    int qp = q_head + lane;
                    if (qp >= kQueueCap) qp -= kQueueCap;
                    rc = fq.rec[qp];
                    if constexpr (kRlo) rl = fq.rlo[qp];
                    kp = fq.rev[qp];
                }
                const int2 done =
                    run_batch(g0 + a_q, na, p, tiv, g0 + a_q + lane, rc, rl, kp, [](int, int) {}, []() {});
                a_q += done.x;
                q_len -= done.y;
                q_head += done.y;
                if (q_head >= kQueueCap) q_head -= kQueueCap;
            }
            if (lane < gn) a.kmask[g0 + lane] = kb;
        }
    }

    if constexpr (BATCHED) return;
    store_partials(a, e_acc, w_acc, n_pairs, n_trip, asym);
}

// ------------------------------------------ lane-per-triplet (comparison) -
//
// The third way to map the triplet loop onto a wavefront (Section 3 weighs
// vectorising over centres and over neighbours; here the lanes take the
// triplets themselves).  Same batches of packed slots, records and outputs as
// k_tersoff, with the work of a batch split by lanes as:
//   slot lanes     record, r_ij, u_ij and f_C of each slot;
//   triplet lanes  the term f_C(r_ik) g(theta_ijk) e(r_ij, r_ik) of zeta_ij,
//                  added into the slot's zeta in LDS (atomics), and the
//                  triplet's derivatives with respect to x_j and x_k;
//   slot lanes     Eq. (2) of the pair: energy, pair force, dV/dzeta_ij;
//   triplet lanes  -dV/dzeta_ij times those derivatives, added (FP64 LDS
//                  atomics) into the forces of slots j and k;
//   slot lanes     virial and the force-plane store; atom lanes the centre's
//                  own force (minus the sum over its slots).
// A lane keeps the derivatives of its first kTripKeep triplets of a batch in
// registers and forms those of later triplets again.  The atomics leave the
// order of the LDS sums, hence their last bits, free from run to run: this
// mapping is a comparison point, not the default.
constexpr int kTripKeep = 4;

template <typename real>
struct TripShared {
    int ti[kWave];
    int cid[kWave];              // atom index of each centre of the batch
    int pcnt[kWave];
    int pstart[kWave + 1];       // first slot of each centre atom
    int tstart[kWave + 1];       // first triplet of each centre atom
    unsigned char owner[kScap];
    double fs[kScap][3];         // triplet forces on each slot's atom, then the slot's total
    real ux[kScap], uy[kScap], uz[kScap], r[kScap];
    real zeta[kScap], dzeta[kScap];
    int mask[kScap];
    real fc[kMaxTypes][kScap], dfc[kMaxTypes][kScap];
};

// floor(x / d) for 0 <= x < 2^11 and 1 <= d <= 64: (x + 1/2) / d lies at
// least 1/(2d) from every integer, far beyond the rounding of one FP32
// reciprocal and product (relative 2^-22, absolute below 2^-10 here).
__device__ __forceinline__ int small_div(int x, int d)
{
    return (int)(((float)x + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

template <typename real>
__global__ __launch_bounds__(kWave) void k_tersoff_trip(ComputeLaunch a, DeviceTable tab)
{
    constexpr bool kRlo = sizeof(real) == 4;
    __shared__ TripShared<real> sh;
    __shared__ TripParam<real> tp[kMaxTypes * kMaxTypes * kMaxTypes];
    const int lane = threadIdx.x;
    const ParamR<real> *ptab = table_r<real>(tab);
    const Rec<real> *recs = static_cast<const Rec<real> *>(a.recs);
    const int nt = tab.ntypes;
    for (int e = lane; e < nt * nt * nt; e += kWave) tp[e] = trip_of(ptab[e]);

    double e_acc = 0.0;
    double w_acc[6] = {0, 0, 0, 0, 0, 0};
    int n_pairs = 0, n_trip = 0;
    bool asym = false;

    // Triplet t of the batch: centre (binary search of the triplet starts),
    // slots j and k (t's place among the centre's p (p - 1) ordered pairs of
    // distinct slots), the term of zeta_ij and its derivatives with respect to
    // x_j and x_k.  False when k is not a third atom of pair (i, j) or (i, j)
    // is no bonded pair: then the triplet contributes nothing.
    auto triplet = [&](int t, int cut, int &sj, int &sk, real &z, real dzj[3], real dzk[3]) -> bool {
        int lo = 0, hi = cut - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sh.tstart[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int al = lo, pm1 = sh.pcnt[al] - 1, loc = t - sh.tstart[al];
        const int jl = small_div(loc, pm1), kk = loc - jl * pm1;
        sj = sh.pstart[al] + jl;
        sk = sh.pstart[al] + kk + (kk >= jl ? 1 : 0);
        const int mj = sh.mask[sj], mk = sh.mask[sk];
        const int ti = sh.ti[al], tj = rec_type(mj), tk = rec_type(mk);
        if (!((mj >> kPairBit) & 1) || !((mk >> (kThirdBit + tj)) & 1)) return false;
        const TripParam<real> q = tp[(ti * nt + tj) * nt + tk];
        const real rj = sh.r[sj], rk = sh.r[sk];
        const real uj[3] = {sh.ux[sj], sh.uy[sj], sh.uz[sj]};
        const real uk[3] = {sh.ux[sk], sh.uy[sk], sh.uz[sk]};
        const real cs = uj[0] * uk[0] + uj[1] * uk[1] + uj[2] * uk[2];
        const Angular<real> an = angular(q, cs);
        real ex, dex;
        exp_term(q, rj, rk, ex, dex);
        const real fck = sh.fc[tj][sk], dfck = sh.dfc[tj][sk];
        z = fck * an.g * ex;
        // d cos / d x_j = (u_k - cos u_j) / r_j, d cos / d x_k = (u_j - cos u_k) / r_k;
        // the exponential factor moves with r_j as dex and with r_k as -dex
        const real w = fck * an.dg * ex;
        const real aj = w * M<real>::rcp(rj), bj = fck * an.g * dex;
        const real ak = w * M<real>::rcp(rk), bk = an.g * (dfck * ex - fck * dex);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dzj[c] = aj * (uk[c] - cs * uj[c]) + bj * uj[c];
            dzk[c] = ak * (uj[c] - cs * uk[c]) + bk * uk[c];
        }
        return true;
    };
    auto scatter = [&](int sj, int sk, const real dzj[3], const real dzk[3]) {
        const real dz = sh.dzeta[sj];
        if (dz == real(0)) return;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            atomicAdd(&sh.fs[sj][c], (double)(-dz * dzj[c]));
            atomicAdd(&sh.fs[sk][c], (double)(-dz * dzk[c]));
        }
    };

    const int B = a.atoms_per_batch;
    const int n = a.n;
    const int ngroups = (n + B - 1) / B;
    const ItemRange items = xcd_items(ngroups);
    for (int grp = items.begin; grp < items.end; grp += items.stride) {
        const int g_end = min((grp + 1) * B, n);
        size_t rec0 = (size_t)grp * B * kRecCap;   // records of a group: in batch order
        for (int a0 = grp * B; a0 < g_end;) {
            // ---- batch: the leading atoms whose slots fit one per lane
            const int nb = g_end - a0;
            int p = 0, tiv = 0, cid = 0;
            if (lane < nb) {
                cid = a0 + lane;
                p = a.pcount[cid];
                tiv = nt == 1 ? 0 : a.types[cid];
            }
            const int ip = wave_incl_scan(p);
            const int cut = __popcll(__ballot(lane < nb && ip <= kScap));   // >= 1: p <= kRecCap
            const int it = wave_incl_scan(lane < cut ? p * (p - 1) : 0);
            if (lane < cut) {
                sh.ti[lane] = tiv;
                sh.cid[lane] = cid;
                sh.pcnt[lane] = p;
                sh.pstart[lane + 1] = ip;
                sh.tstart[lane + 1] = it;
                for (int q = ip - p; q < ip; ++q) sh.owner[q] = (unsigned char)lane;
            }
            if (lane == 0) {
                sh.pstart[0] = 0;
                sh.tstart[0] = 0;
            }
            const int npacked = __shfl(ip, cut - 1, kWave);
            const int T = __shfl(it, cut - 1, kWave);
            __syncthreads();

            // ---- slot lanes
            const int s = lane;
            const bool has_slot = s < npacked;
            int al = 0, j = 0, kpos = -1, mj = 0, ti = 0;
            real rj = 0, rjlo = 0, uj[3] = {0, 0, 0}, dj[3] = {0, 0, 0};
            if (has_slot) {
                al = sh.owner[s];
                ti = sh.ti[al];
                const Rec<real> rc = recs[rec0 + s];
                if constexpr (kRlo) rjlo = a.rlo[rec0 + s];
                j = rc.jm & kIdMask;
                bool absent;
                kpos = kept_position(a.kept, a.kept + (size_t)kKeptFast * a.plane_stride, j, sh.cid[al], absent);
                asym |= absent;
                mj = rc.jm;
                dj[0] = rc.dx; dj[1] = rc.dy; dj[2] = rc.dz;
                rj = M<real>::sqrt(norm2r(dj[0], dj[1], dj[2]));
                const real rinv = M<real>::rcp(rj);
                uj[0] = dj[0] * rinv; uj[1] = dj[1] * rinv; uj[2] = dj[2] * rinv;
                sh.ux[s] = uj[0]; sh.uy[s] = uj[1]; sh.uz[s] = uj[2];
                sh.r[s] = rj;
                sh.mask[s] = mj;
                for (int t = 0; t < nt; ++t) {
                    real fc = real(0), dfc = real(0);
                    if ((mj >> (kThirdBit + t)) & 1)
                        cutoff_terms(ptab[(ti * nt + t) * nt + rec_type(mj)], rj, fc, dfc, rjlo);
                    sh.fc[t][s] = fc;
                    sh.dfc[t][s] = dfc;
                }
                sh.zeta[s] = real(0);
                sh.fs[s][0] = 0.0; sh.fs[s][1] = 0.0; sh.fs[s][2] = 0.0;
            }
            __syncthreads();

            // ---- triplet lanes: zeta_ij, and the derivatives of each term
            int keep_s[kTripKeep];
            real keep_j[kTripKeep][3], keep_k[kTripKeep][3];
#pragma unroll
            for (int q = 0; q < kTripKeep; ++q) {
                keep_s[q] = -1;
                const int t = q * kWave + lane;
                int sj, sk;
                real z;
                if (t < T && triplet(t, cut, sj, sk, z, keep_j[q], keep_k[q])) {
                    ++n_trip;
                    keep_s[q] = sj | (sk << 8);
                    atomicAdd(&sh.zeta[sj], z);
                }
            }
            for (int t = kTripKeep * kWave + lane; t < T; t += kWave) {
                int sj, sk;
                real z, vj[3], vk[3];
                if (triplet(t, cut, sj, sk, z, vj, vk)) {
                    ++n_trip;
                    atomicAdd(&sh.zeta[sj], z);
                }
            }
            __syncthreads();

            // ---- slot lanes: Eq. (2) of the pair
            const int tj = rec_type(mj);
            double fx = 0, fy = 0, fz = 0, e_pair = 0.0;
            if (has_slot) {
                real dz_out = real(0);
                if ((mj >> kPairBit) & 1) {
                    ++n_pairs;
                    const int e_ij = (ti * nt + tj) * nt + tj;
                    pair_step<real, false>(ptab[e_ij], tab.px[e_ij], sh.zeta[s], sh.fc[tj][s], sh.dfc[tj][s], rj,
                                           rjlo, uj, e_pair, dz_out, fx, fy, fz);
                    e_acc += e_pair;
                }
                sh.dzeta[s] = dz_out;
            }
            __syncthreads();

            // ---- triplet lanes: the force terms of every triplet on j and k
#pragma unroll
            for (int q = 0; q < kTripKeep; ++q)
                if (keep_s[q] >= 0) scatter(keep_s[q] & 255, keep_s[q] >> 8, keep_j[q], keep_k[q]);
            for (int t = kTripKeep * kWave + lane; t < T; t += kWave) {
                int sj, sk;
                real z, vj[3], vk[3];
                if (triplet(t, cut, sj, sk, z, vj, vk)) scatter(sj, sk, vj, vk);
            }
            __syncthreads();

            // ---- slot lanes: total force of centre i on j, virial, plane store
            if (has_slot) {
                const double Fx = fx + sh.fs[s][0], Fy = fy + sh.fs[s][1], Fz = fz + sh.fs[s][2];
                const double dxj = (double)dj[0], dyj = (double)dj[1], dzj = (double)dj[2];
                w_acc[0] += dxj * Fx;
                w_acc[1] += dyj * Fy;
                w_acc[2] += dzj * Fz;
                w_acc[3] += dxj * Fy;
                w_acc[4] += dxj * Fz;
                w_acc[5] += dyj * Fz;
                if ((unsigned)kpos < (unsigned)kRecCap) {
                    real *f = static_cast<real *>(a.planes) + 3 * ((size_t)kpos * a.plane_stride + (size_t)j);
                    f[0] = (real)Fx; f[1] = (real)Fy; f[2] = (real)Fz;
                }
                sh.fs[s][0] = Fx; sh.fs[s][1] = Fy; sh.fs[s][2] = Fz;
            }
            __syncthreads();
            if (lane < cut) {
                double ox = 0, oy = 0, oz = 0;
                for (int q = sh.pstart[lane]; q < sh.pstart[lane + 1]; ++q) {
                    ox -= sh.fs[q][0]; oy -= sh.fs[q][1]; oz -= sh.fs[q][2];
                }
                double *o = a.own + 3 * (size_t)cid;
                o[0] = ox; o[1] = oy; o[2] = oz;
            }
            __syncthreads();
            a0 += cut;
            rec0 += npacked;
        }
    }
    store_partials(a, e_acc, w_acc, n_pairs, n_trip, asym);
}

// Atoms dropped by k_pack (more kept neighbours than a record row holds) are
// evaluated with a truncated neighbour set and reported invalid; zero the
// force slots their neighbours reserved for them so the gather adds nothing
// from them.  Workgroups loop until the list is
// drained.
template <typename T>
__global__ void k_fixup_dropped(const int *__restrict__ ell, int cap, const int *__restrict__ row_count,
                                const int *__restrict__ kept, const int *__restrict__ kept_more,
                                const int *__restrict__ drop_list, const int *__restrict__ drop_count,
                                int plane_stride, T *__restrict__ planes)
{
    const int nd = *drop_count;
    for (int q = blockIdx.x; q < nd; q += gridDim.x) {
        const int m = drop_list[q];
        const int rc = row_count[m];
        for (int q = (int)threadIdx.x; q < rc; q += blockDim.x) {
            const int nb = ell[(size_t)m * cap + q];
            bool absent;
            const int k = kept_position(kept, kept_more, nb, m, absent);   // plane nb reserved for m
            if (k >= 0) {
                T *f = planes + 3 * ((size_t)k * plane_stride + (size_t)nb);
                f[0] = f[1] = f[2] = T(0);
            }
        }
    }
}

// Sums the per-workgroup partials of the compute kernel in one workgroup of
// NT threads (fixed summation order: each thread its rows t, t + NT, ...,
// then a butterfly within each wavefront, then the wavefront sums in order)
// and raises kFlagAsym if a workgroup reported it.
template <int NT>
__device__ __forceinline__ void finalize_sums(const double *__restrict__ partials,
                                              const long long *__restrict__ counters, int grid,
                                              double *__restrict__ out, long long *__restrict__ counts, int *flags)
{
    __shared__ double sh[NT / kWave][7];
    __shared__ long long shc[NT / kWave][2];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    long long c0 = 0, c1 = 0;
    bool asym = false;
    // the loads of four rows are issued before their sums
    constexpr int kU = 4;
    for (int b0 = threadIdx.x; b0 < grid; b0 += kU * NT) {
        double pr[kU][8];
        long long cr[kU][2];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int b = min(b0 + u * NT, grid - 1);
#pragma unroll
            for (int c = 0; c < 8; ++c) pr[u][c] = partials[8 * (size_t)b + c];
            cr[u][0] = counters[2 * (size_t)b];
            cr[u][1] = counters[2 * (size_t)b + 1];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (b0 + u * NT >= grid) break;
#pragma unroll
            for (int c = 0; c < 7; ++c) v[c] += pr[u][c];
            asym |= pr[u][7] != 0.0;
            c0 += cr[u][0];
            c1 += cr[u][1];
        }
    }
    if (asym) atomicOr(flags, kFlagAsym);
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = wave_sum(v[c]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        c0 += __shfl_xor(c0, off, kWave);
        c1 += __shfl_xor(c1, off, kWave);
    }
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
#pragma unroll
        for (int c = 0; c < 7; ++c) sh[w][c] = v[c];
        shc[w][0] = c0;
        shc[w][1] = c1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[7] = {0, 0, 0, 0, 0, 0, 0};
        long long n0 = 0, n1 = 0;
        for (int q = 0; q < NT / kWave; ++q) {
#pragma unroll
            for (int c = 0; c < 7; ++c) t[c] += sh[q][c];
            n0 += shc[q][0];
            n1 += shc[q][1];
        }
#pragma unroll
        for (int c = 0; c < 7; ++c) out[c] = t[c];
        counts[0] = n0;
        counts[1] = n1;
    }
}

// One workgroup per system of a batch: sums of the per-atom energy and
// virial over the system's atoms (thread t takes local atoms t, t + 256, ...,
// then a fixed tree), so a system's result does not depend on where in the
// batch it sits; status bits from the search and the dropped-atom list.
__global__ void k_reduce_systems(const SysDesc *__restrict__ sys, const BatchDims *__restrict__ dims,
                                 const double *__restrict__ eatom, const int *__restrict__ drop_list,
                                 const int *__restrict__ drop_count, const int *__restrict__ sys_status,
                                 double *__restrict__ out)
{
    __shared__ double sh[7][256];
    const int nsys = dims->n_sys;
    const int nd = *drop_count;
    for (int s = blockIdx.x; s < nsys; s += gridDim.x) {
        const int a0 = sys[s].atom_off, na = sys[s].natoms;
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int k = threadIdx.x; k < na; k += blockDim.x)
            #pragma unroll
            for (int c = 0; c < 7; ++c) v[c] += eatom[8 * (size_t)(a0 + k) + c];
        #pragma unroll
        for (int c = 0; c < 7; ++c) sh[c][threadIdx.x] = v[c];
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off)
                #pragma unroll
                for (int c = 0; c < 7; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            int st = sys_status[s];
            for (int q = 0; q < nd; ++q)
                if (drop_list[q] >= a0 && drop_list[q] < a0 + na) st |= 2;
            #pragma unroll
            for (int c = 0; c < 7; ++c) out[8 * (size_t)s + c] = sh[c][0];
            out[8 * (size_t)s + 7] = (double)st;
        }
        __syncthreads();
    }
}

// F_m = (terms of centre m) + the force each centre i that keeps m put into
// plane k of m, k = rank of i among m's kept neighbours (k < pcount[m]),
// stored at forces[perm[m]] (perm: the caller's index of each atom of the
// internal numbering; null: the same numbering).
// One thread per atom; each plane read is coalesced across the wavefront.
// Also empties the dropped-atom list for the next evaluation when
// drop_count is given (every kernel reading it has run by now), and, when
// fin.partials is given, sums the compute kernel's partials in one extra
// workgroup -- the first, so that it runs beside the gather rather than
// after it.
template <typename T>
__global__ __launch_bounds__(kGatherThreads) void k_gather_forces(const int *__restrict__ pcount,
                                                                  const T *__restrict__ planes,
                                                                  const double *__restrict__ own, int n,
                                                                  const int *__restrict__ n_dev, int plane_stride,
                                                                  double *__restrict__ forces,
                                                                  const int *__restrict__ perm, int *drop_count,
                                                                  FinalizeArgs fin)
{
    if (fin.partials && blockIdx.x == 0) {
        finalize_sums<kGatherThreads>(fin.partials, fin.counters, fin.grid, fin.out, fin.counts, fin.flags);
        return;
    }
    const int blk = blockIdx.x - (fin.partials ? 1 : 0);
    if (drop_count && blk == 0 && threadIdx.x == 0) *drop_count = 0;
    const int m = blk * (int)blockDim.x + (int)threadIdx.x;
    if (m >= (n_dev ? *n_dev : n)) return;
    double fx = own[3 * (size_t)m], fy = own[3 * (size_t)m + 1], fz = own[3 * (size_t)m + 2];
    const int pc = pcount[m];
    // planes 0 .. pc-1 in order; the loads of four planes are issued together
    for (int k0 = 0; k0 < pc; k0 += 4) {
        T v[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T *f = planes + 3 * ((size_t)min(k0 + u, pc - 1) * plane_stride + (size_t)m);
            v[u][0] = f[0];
            v[u][1] = f[1];
            v[u][2] = f[2];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (k0 + u >= pc) break;
            fx += (double)v[u][0];
            fy += (double)v[u][1];
            fz += (double)v[u][2];
        }
    }
    const size_t o = perm ? (size_t)perm[m] : (size_t)m;
    forces[3 * o] = fx;
    forces[3 * o + 1] = fy;
    forces[3 * o + 2] = fz;
}

// Fused packing: F_m = (terms of centre m) + plane e of m for every row
// position e whose centre keeps m (kmask[m]), in increasing e; the centre at
// row position e of m wrote its force on m there (or zero when m was beyond
// its slots).  Partials and perm as k_gather_forces.
template <typename T>
__global__ __launch_bounds__(kGatherThreads) void k_gather_rows(const unsigned long long *__restrict__ kmask,
                                                                const T *__restrict__ planes,
                                                                const double *__restrict__ own, int n,
                                                                int plane_stride, double *__restrict__ forces,
                                                                const int *__restrict__ perm, FinalizeArgs fin)
{
    if (fin.partials && blockIdx.x == 0) {
        finalize_sums<kGatherThreads>(fin.partials, fin.counters, fin.grid, fin.out, fin.counts, fin.flags);
        return;
    }
    const int blk = blockIdx.x - (fin.partials ? 1 : 0);
    const int m = blk * (int)blockDim.x + (int)threadIdx.x;
    if (m >= n) return;
    double fx = own[3 * (size_t)m], fy = own[3 * (size_t)m + 1], fz = own[3 * (size_t)m + 2];
    unsigned long long bits = kmask[m];
    // four planes' loads issued together
    while (bits) {
        int e[4], cnt = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            e[u] = bits ? __builtin_ctzll(bits) : e[0];
            if (bits) {
                bits &= bits - 1;
                ++cnt;
            }
        }
        T v[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T *f = planes + 3 * ((size_t)e[u] * plane_stride + (size_t)m);
            v[u][0] = f[0];
            v[u][1] = f[1];
            v[u][2] = f[2];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (u >= cnt) break;
            fx += (double)v[u][0];
            fy += (double)v[u][1];
            fz += (double)v[u][2];
        }
    }
    const size_t o = perm ? (size_t)perm[m] : (size_t)m;
    forces[3 * o] = fx;
    forces[3 * o + 1] = fy;
    forces[3 * o + 2] = fz;
}

// One thread per row entry (i, e): the position of i in the row of its
// neighbour (binary search of the sorted row).
__global__ void k_reverse_index(const int *__restrict__ ell, const int *__restrict__ row_count, int cap, int n,
                                unsigned char *__restrict__ rev, int *flags)
{
    const size_t total = (size_t)n * cap;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / cap), e = (int)(q % cap);
        if (e >= min(row_count[i], cap)) continue;
        const int j = ell[q];
        const int *row = ell + (size_t)j * cap;
        int lo = 0, hi = min(row_count[j], cap);   // first position with row[pos] >= i
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (row[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        int pos = lo;
        if (lo >= min(row_count[j], cap) || row[lo] != i) {
            atomicOr(flags, kFlagAsym);
            pos = 0;
        }
        rev[q] = (unsigned char)pos;
    }
}

template <typename T>
__global__ void k_fill_zero(T *p, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = T(0);
}

// Workgroups of a persistent grid: the resident limit per CU (at most
// max_per_cu) times the CU count, at most one per work item.
// Resident workgroups per CU of a kernel and the device's CU count, queried
// once per (device, kernel) and kept: every build sizes its grids from them.
int occupancy_grid(const void *kern, long long work_items, int max_per_cu = 1 << 20)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, std::pair<int, int>> known;
    int dev = 0;
    (void)hipGetDevice(&dev);
    int per_cu = 0, cus = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = known.find({dev, kern});
        if (it != known.end()) {
            per_cu = it->second.first;
            cus = it->second.second;
        }
    }
    if (cus == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kWave, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        cus = 256;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        std::lock_guard<std::mutex> lock(mu);
        known[{dev, kern}] = {per_cu, cus};
    }
    per_cu = std::min(per_cu, max_per_cu);
    long long g = (long long)per_cu * cus;
    if (g > work_items) g = work_items;
    return (int)(g < 1 ? 1 : g);
}

// Instances of the compute kernel: precision x kind.  Kind 0: up to
// kMaxTypes species, any table; 1: one species; 2: one species without the
// lambda3 term (lambda3 = 0); 3: up to two species whose three-body
// parameters are symmetric in j and k (the k-role terms cached).
template <typename T>
struct TypeTag {
    using type = T;
};
template <typename R, int NT_, bool S, bool N, bool C>
struct KernelTag {
    using real = R;
    static constexpr int nt = NT_;
    static constexpr bool one = NT_ == 1, single = S, nol3 = N, cache = C;
};

int table_kind(const DeviceTable &t)
{
    if (t.ntypes == 1) return t.lam3_zero ? 2 : 1;
    return (t.ntypes == 2 && t.sym3) ? 3 : 0;
}

template <typename F>
void with_kernel(int prec, int kind, F &&f)
{
    auto by_kind = [&](auto r_tag, auto s_tag) {
        using R = typename decltype(r_tag)::type;
        constexpr bool S = decltype(s_tag)::value;
        if (kind == 0) f(KernelTag<R, kMaxTypes, S, false, false>{});
        else if (kind == 1) f(KernelTag<R, 1, S, false, true>{});
        else if (kind == 2) f(KernelTag<R, 1, S, true, true>{});
        else f(KernelTag<R, 2, S, false, true>{});
    };
    if (prec == kPrecSingle) by_kind(TypeTag<float>{}, std::true_type{});
    else if (prec == kPrecMixed) by_kind(TypeTag<float>{}, std::false_type{});
    else by_kind(TypeTag<double>{}, std::false_type{});
}

template <bool BATCHED>
void grids_dispatch(int prec, const DeviceTable &t, int n, int atoms_per_batch, int grids[4])
{
    const long long batches = ((long long)n + atoms_per_batch - 1) / atoms_per_batch;
    with_kernel(prec, table_kind(t), [&](auto tag) {
        using K = decltype(tag);
        grids[0] = occupancy_grid((const void *)k_pack<typename K::real, K::one, BATCHED>, batches,
                                  kPackWavesPerCU);
        grids[1] = occupancy_grid(
            (const void *)k_tersoff<typename K::real, K::nt, BATCHED, K::single, K::nol3, K::cache>, batches,
            kComputeWavesPerCU[prec]);
        grids[3] = BATCHED ? 0
                           : occupancy_grid((const void *)k_tersoff<typename K::real, K::nt, false, K::single, K::nol3,
                                                                    K::cache, false, true>,
                                            batches, kComputeWavesPerCU[prec]);
    });
    grids[2] = kBigGrid;
}

template <bool BATCHED>
void pack_dispatch(const PackLaunch &a, const DeviceTable &t, int prec, int grid, hipStream_t s)
{
    const bool one = t.ntypes == 1;
    if (prec != kPrecFP64) {
        if (one) hipLaunchKernelGGL((k_pack<float, true, BATCHED>), dim3(grid), dim3(kWave), 0, s, a, t);
        else hipLaunchKernelGGL((k_pack<float, false, BATCHED>), dim3(grid), dim3(kWave), 0, s, a, t);
    } else {
        if (one) hipLaunchKernelGGL((k_pack<double, true, BATCHED>), dim3(grid), dim3(kWave), 0, s, a, t);
        else hipLaunchKernelGGL((k_pack<double, false, BATCHED>), dim3(grid), dim3(kWave), 0, s, a, t);
    }
}

template <bool BATCHED>
void compute_dispatch(const ComputeLaunch &a, const DeviceTable &t, int prec, int grid, hipStream_t s)
{
    const dim3 G(grid), W(kWave);
    with_kernel(prec, table_kind(t), [&](auto tag) {
        using K = decltype(tag);
        if constexpr (!BATCHED) {
            if (a.rows) {
                hipLaunchKernelGGL(
                    (k_tersoff<typename K::real, K::nt, false, K::single, K::nol3, K::cache, false, true>), G, W, 0,
                    s, a, t);
                return;
            }
            if (a.forces_atomic) {
                hipLaunchKernelGGL((k_tersoff<typename K::real, K::nt, false, K::single, K::nol3, K::cache, true>), G,
                                   W, 0, s, a, t);
                return;
            }
        }
        hipLaunchKernelGGL((k_tersoff<typename K::real, K::nt, BATCHED, K::single, K::nol3, K::cache>), G, W, 0, s,
                           a, t);
    });
}

}  // namespace

void compute_grids(int prec, const DeviceTable &t, bool batched, int n, int atoms_per_batch, int grids[4])
{
    if (batched) grids_dispatch<true>(prec, t, n, atoms_per_batch, grids);
    else grids_dispatch<false>(prec, t, n, atoms_per_batch, grids);
}

size_t record_bytes(int prec) { return prec != kPrecFP64 ? sizeof(Rec<float>) : sizeof(Rec<double>); }

size_t record_region_bytes(int prec, size_t slots)
{
    return prec != kPrecFP64 ? slots * (sizeof(Rec<float>) + sizeof(float)) : slots * sizeof(Rec<double>);
}

float *rlo_of(void *recs, int prec, size_t slots)
{
    if (prec == kPrecFP64) return nullptr;
    return reinterpret_cast<float *>(static_cast<unsigned char *>(recs) + slots * sizeof(Rec<float>));
}

hipError_t launch_pack(const PackLaunch &a, const DeviceTable &t, int prec, int grid, hipStream_t s)
{
    if (a.n_dev) pack_dispatch<true>(a, t, prec, grid, s);
    else pack_dispatch<false>(a, t, prec, grid, s);
    return hipGetLastError();
}

hipError_t launch_compute(const ComputeLaunch &a, const DeviceTable &t, int prec, int grid,
                          hipStream_t s)
{
    if (a.atoms_per_batch < 1 || a.atoms_per_batch > kWave) return hipErrorInvalidValue;
    if (a.n_dev) compute_dispatch<true>(a, t, prec, grid, s);
    else compute_dispatch<false>(a, t, prec, grid, s);
    return hipGetLastError();
}

hipError_t launch_compute_triplet(const ComputeLaunch &a, const DeviceTable &t, int prec, int max_grid,
                                  hipStream_t s, int *grid_used)
{
    if (a.n_dev || a.forces_atomic || prec == kPrecSingle || a.atoms_per_batch < 1 || a.atoms_per_batch > kWave ||
        max_grid < 1)
        return hipErrorInvalidValue;
    const long long batches = ((long long)a.n + a.atoms_per_batch - 1) / a.atoms_per_batch;
    const void *k = prec == kPrecMixed ? (const void *)k_tersoff_trip<float> : (const void *)k_tersoff_trip<double>;
    const int g = std::min(max_grid, occupancy_grid(k, batches, kComputeWavesPerCU[prec]));
    if (prec == kPrecMixed) hipLaunchKernelGGL(k_tersoff_trip<float>, dim3(g), dim3(kWave), 0, s, a, t);
    else hipLaunchKernelGGL(k_tersoff_trip<double>, dim3(g), dim3(kWave), 0, s, a, t);
    *grid_used = g;
    return hipGetLastError();
}

hipError_t launch_fixup_dropped(const int *ell, int cap, const int *row_count, const int *kept,
                                const int *kept_more, const int *drop_list, const int *drop_count,
                                int plane_stride, int prec, void *planes, hipStream_t s)
{
    if (prec != kPrecFP64)
        hipLaunchKernelGGL(k_fixup_dropped<float>, dim3(kBigGrid), dim3(kWave), 0, s, ell, cap, row_count, kept,
                           kept_more, drop_list, drop_count, plane_stride, static_cast<float *>(planes));
    else
        hipLaunchKernelGGL(k_fixup_dropped<double>, dim3(kBigGrid), dim3(kWave), 0, s, ell, cap, row_count, kept,
                           kept_more, drop_list, drop_count, plane_stride, static_cast<double *>(planes));
    return hipGetLastError();
}

hipError_t launch_reduce_systems(const SysDesc *sys, const BatchDims *dims, int max_sys, const double *eatom,
                                 const int *drop_list, const int *drop_count, const int *sys_status,
                                 double *out, hipStream_t s)
{
    const int grid = std::max(1, std::min(max_sys, kBatchGrid));
    hipLaunchKernelGGL(k_reduce_systems, dim3(grid), dim3(256), 0, s, sys, dims, eatom, drop_list, drop_count,
                       sys_status, out);
    return hipGetLastError();
}

hipError_t launch_gather_forces(const int *pcount, int prec, const void *planes, const double *own, int n,
                                const int *n_dev, int plane_stride, double *forces, const int *perm,
                                int *drop_count, const FinalizeArgs &fin, hipStream_t s)
{
    const int blocks = std::max(1, (n + kGatherThreads - 1) / kGatherThreads) + (fin.partials ? 1 : 0);
    const dim3 G(blocks), W(kGatherThreads);
    if (prec != kPrecFP64)
        hipLaunchKernelGGL(k_gather_forces<float>, G, W, 0, s, pcount, static_cast<const float *>(planes), own, n,
                           n_dev, plane_stride, forces, perm, drop_count, fin);
    else
        hipLaunchKernelGGL(k_gather_forces<double>, G, W, 0, s, pcount, static_cast<const double *>(planes), own,
                           n, n_dev, plane_stride, forces, perm, drop_count, fin);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const unsigned long long *kmask, int prec, const void *planes, const double *own,
                              int n, int plane_stride, double *forces, const int *perm, const FinalizeArgs &fin,
                              hipStream_t s)
{
    const int blocks = std::max(1, (n + kGatherThreads - 1) / kGatherThreads) + (fin.partials ? 1 : 0);
    const dim3 G(blocks), W(kGatherThreads);
    if (prec != kPrecFP64)
        hipLaunchKernelGGL(k_gather_rows<float>, G, W, 0, s, kmask, static_cast<const float *>(planes), own, n,
                           plane_stride, forces, perm, fin);
    else
        hipLaunchKernelGGL(k_gather_rows<double>, G, W, 0, s, kmask, static_cast<const double *>(planes), own, n,
                           plane_stride, forces, perm, fin);
    return hipGetLastError();
}

hipError_t launch_reverse_index(const int *ell, const int *row_count, int cap, int n, unsigned char *rev,
                                int *flags, hipStream_t s)
{
    const long long total = (long long)n * cap;
    const int grid = (int)std::max(1LL, std::min((total + 255) / 256, 8192LL));
    hipLaunchKernelGGL(k_reverse_index, dim3(grid), dim3(256), 0, s, ell, row_count, cap, n, rev, flags);
    return hipGetLastError();
}

// Positions in the internal numbering: posp[t] = pos[perm[t]]; and back:
// out[perm[t]] = in[t] (three doubles per atom each).
__global__ void k_unpermute3(const double *__restrict__ in, const int *__restrict__ perm, int n,
                             double *__restrict__ out)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const size_t i = (size_t)perm[t];
        out[3 * i] = in[3 * (size_t)t];
        out[3 * i + 1] = in[3 * (size_t)t + 1];
        out[3 * i + 2] = in[3 * (size_t)t + 2];
    }
}

hipError_t launch_unpermute3(const double *in, const int *perm, int n, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = std::max(1, std::min((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_unpermute3, dim3(grid), dim3(256), 0, s, in, perm, n, out);
    return hipGetLastError();
}

__global__ void k_permute_pos(const double *__restrict__ pos, const int *__restrict__ perm, int n,
                              double *__restrict__ posp)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const size_t i = (size_t)perm[t];
        posp[3 * (size_t)t] = pos[3 * i];
        posp[3 * (size_t)t + 1] = pos[3 * i + 1];
        posp[3 * (size_t)t + 2] = pos[3 * i + 2];
    }
}

hipError_t launch_permute_pos(const double *pos, const int *perm, int n, double *posp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = std::max(1, std::min((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_permute_pos, dim3(grid), dim3(256), 0, s, pos, perm, n, posp);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *p, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero<double>, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_fill_zero_int(int *p, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero<int>, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

}  // namespace tsf
