// Tersoff energy / force / virial kernel (Eq. 1-3, Algorithm 1).
//
// One 64-lane wavefront per workgroup walks batches of consecutive centre
// atoms.  Each batch goes through five phases, every phase with its lanes
// mapped to a different kind of work item, so that the short in-cutoff lists
// of a many-body potential do not leave lanes idle (the problem of Section 2;
// Section 3 packs the in-cutoff entries and vectorises over (i, j) pairs):
//
//   A  lanes = list entries of the batch's atoms (contiguous CSR range):
//      FP64 minimum-image displacement, r^2, skin exclusion; the entries
//      inside the interaction range are packed (ballot + prefix count) into
//      LDS slots, grouped by centre atom, with r, 1/r and the unit vector.
//   C  lanes = ordered triplets (i; j, k != j) of packed slots: zeta(i,j,k)
//      and its gradients d zeta / d x_j, d zeta / d x_k (computed once and
//      kept in registers for the second K loop); zeta_ij summed per slot by
//      LDS atomics.
//   D  lanes = packed slots (i, j): f_C, f_R, f_A, the bond order b_ij and
//      db/dzeta in FP64 log form, energy, pair force, dV/dzeta.
//   E  lanes = triplets again: dV/dzeta * gradients, accumulated per slot and
//      per centre atom in LDS (FP64).
//   F  one FP64 global atomic triple per slot and per centre atom.
//
// `real` is float for the mixed path and double for the all-FP64 path; the
// displacement, the zeta -> b power and every accumulation are FP64 in both.
#include "internal.h"

#include <cmath>

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
    static __device__ __forceinline__ void sincos(float x, float *s, float *c) { ::sincosf(x, s, c); }
};

template <>
struct M<double> {
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ void sincos(double x, double *s, double *c) { ::sincos(x, s, c); }
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

// ------------------------------------------------------------ parameters --

template <typename real>
__device__ __forceinline__ const ParamR<real> *table_r(const DeviceTable &t);
template <>
__device__ __forceinline__ const ParamR<float> *table_r<float>(const DeviceTable &t) { return t.pf; }
template <>
__device__ __forceinline__ const ParamR<double> *table_r<double>(const DeviceTable &t) { return t.pd; }

// ------------------------------------------------------------- LDS layout -

template <typename real, int SCAP>
struct Shared {
    // per centre atom of the batch
    double xi[kWave], yi[kWave], zi[kWave];
    double fi[kWave][3];
    int ti[kWave];
    int eoff[kWave + 1];
    int pcnt[kWave];
    int pstart[kWave + 1];
    int tstart[kWave + 1];
    // per packed slot (i, n)
    double rsq[SCAP];
    double fs[SCAP][3];      // force on atom n accumulated in this batch
    real ux[SCAP], uy[SCAP], uz[SCAP];
    real r[SCAP], rinv[SCAP];
    real zeta[SCAP];
    real dzeta[SCAP];        // dV(i,n,zeta)/dzeta
    int j[SCAP];
    int e[SCAP];             // entry (j, i) of the slot's reverse pair
    int tj[SCAP];
    int al[SCAP];            // centre atom (batch-local)
};

// f_R = A exp(-lambda1 r), f_A = -B exp(-lambda2 r) and their derivatives.
// FP64: direct.  FP32: exp(ln A - lambda1 r) with the argument carried as an
// unevaluated float pair (two-sum and fma error terms), so the rounding of
// A and lambda1 to float leaves no systematic bias in the pair energy.
__device__ __forceinline__ float exp_compensated(float a, float a_lo, float l, float l_lo, float r)
{
    const float p = l * r;
    const float pe = fmaf(l, r, -p);            // l r = p + pe exactly
    const float s = a - p;                      // two-sum of a and -p
    const float bb = s - a;
    const float e = (a - (s - bb)) + (-p - bb);
    const float lo = ((e + a_lo) - pe) - l_lo * r;
    const float x = expf(s);
    return fmaf(x, lo, x);
}

__device__ __forceinline__ void pair_terms(const ParamR<float> &q, float r, float &fr, float &dfr,
                                           float &fa, float &dfa)
{
    fr = exp_compensated(q.lnA, q.lnA_lo, q.lam1, q.lam1_lo, r);
    fa = -exp_compensated(q.lnB, q.lnB_lo, q.lam2, q.lam2_lo, r);
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

// Switching function f_C(r) and its derivative.  r - R is exact in the
// switching zone (Sterbenz), and the rounding errors of R and pi/(2D) in the
// working precision are added back, so f_C carries no systematic bias.
template <typename real>
__device__ __forceinline__ void cutoff_terms(const ParamR<real> &q, real r, real &fc, real &dfc)
{
    fc = real(1);
    dfc = real(0);
    if (r >= q.Rin) {
        const real dr = (r - q.R) - q.R_lo;
        const real arg = dr * q.half_pi_D + dr * q.half_pi_D_lo;
        real sn, cn;
        M<real>::sincos(arg, &sn, &cn);
        fc = real(0.5) - real(0.5) * sn;
        dfc = real(-0.5) * (q.half_pi_D + q.half_pi_D_lo) * cn;
    }
}

// zeta(i,j,k) and its gradients with respect to x_j and x_k.
template <typename real>
struct Trip {
    real z;
    real gj[3], gk[3];
};

template <typename real, bool GRAD>
__device__ __forceinline__ void triplet_term(const ParamR<real> &q, real rj, real rjinv,
                                             const real uj[3], real rk, real rkinv,
                                             const real uk[3], Trip<real> &o)
{
    const real one = real(1);
    real cs = uj[0] * uk[0] + uj[1] * uk[1] + uj[2] * uk[2];
    // cutoff function of r_ik
    real fc, dfc;
    cutoff_terms(q, rk, fc, dfc);
    // angular term, cancellation-free: g = gamma (1 + (c^2/d^2) t^2 / (d^2 + t^2))
    real t = cs - q.h;
    real den = q.d2 + t * t;
    real iden = M<real>::rcp(den);
    real g = q.gamma * (one + q.c2d2 * t * t * iden);
    // exp((lambda3 (rij - rik))^m)
    real ex = one, dex = real(0);
    if (q.lam3 != real(0)) {
        real dr = rj - rk;
        if (q.m == real(3)) {
            real dr2 = dr * dr;
            ex = M<real>::exp(q.lam3m * dr2 * dr);
            dex = real(3) * q.lam3m * dr2 * ex;
        } else {
            ex = M<real>::exp(q.lam3 * dr);
            dex = q.lam3 * ex;
        }
    }
    o.z = fc * g * ex;
    if (GRAD) {
        real dg = q.gamma * q.two_c2 * t * iden * iden;
        real a = fc * ex * dg;          // multiplies d cos / dx
        real bj = fc * g * dex;         // along u_ij
        real bk = dfc * g * ex - bj;    // along u_ik
        real aj = a * rjinv, ak = a * rkinv;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o.gj[c] = aj * (uk[c] - cs * uj[c]) + bj * uj[c];
            o.gk[c] = ak * (uj[c] - cs * uk[c]) + bk * uk[c];
        }
    }
}

struct TripIdx {
    int al, sj, sk;
};

template <typename real, int SCAP>
__device__ __forceinline__ TripIdx decode_triplet(const Shared<real, SCAP> &sh, int nat, int t)
{
    TripIdx r;
    r.al = find_seg(sh.tstart, nat, t);
    int q = t - sh.tstart[r.al];
    int p1 = sh.pcnt[r.al] - 1;   // >= 1 whenever atom al owns triplets
    // q / p1 by a float reciprocal: q < 2^12, the quotient is never within
    // 1/(2 p1) of an integer boundary, far above the float rounding error.
    int jl = (int)(((float)q + 0.5f) * __builtin_amdgcn_rcpf((float)p1));
    int kl = q - jl * p1;
    kl += (kl >= jl);
    r.sj = sh.pstart[r.al] + jl;
    r.sk = sh.pstart[r.al] + kl;
    return r;
}

template <typename real, bool ONE, int SCAP>
__device__ __forceinline__ bool triplet_eval(const Shared<real, SCAP> &sh, const TripIdx &ix,
                                             const DeviceTable &tab, const ParamR<real> *ptab,
                                             Trip<real> &o, bool grad)
{
    int ti = ONE ? 0 : sh.ti[ix.al];
    int tj = ONE ? 0 : sh.tj[ix.sj];
    int tk = ONE ? 0 : sh.tj[ix.sk];
    int nt = ONE ? 1 : tab.ntypes;
    int e_ij = (ti * nt + tj) * nt + tj;
    int e_ijk = (ti * nt + tj) * nt + tk;
    if (!ONE) {
        // bond (i,j) must be inside its own cutoff, k inside the (i,j,k) cutoff
        if (!(sh.rsq[ix.sj] < tab.px[e_ij].cutsq) || !(sh.rsq[ix.sk] < tab.px[e_ijk].cutsq)) {
            o.z = real(0);
            for (int c = 0; c < 3; ++c) o.gj[c] = o.gk[c] = real(0);
            return false;
        }
    }
    const ParamR<real> &q = ptab[e_ijk];
    real uj[3] = {sh.ux[ix.sj], sh.uy[ix.sj], sh.uz[ix.sj]};
    real uk[3] = {sh.ux[ix.sk], sh.uy[ix.sk], sh.uz[ix.sk]};
    if (grad)
        triplet_term<real, true>(q, sh.r[ix.sj], sh.rinv[ix.sj], uj, sh.r[ix.sk], sh.rinv[ix.sk], uk, o);
    else
        triplet_term<real, false>(q, sh.r[ix.sj], sh.rinv[ix.sj], uj, sh.r[ix.sk], sh.rinv[ix.sk], uk, o);
    return true;
}

// ------------------------------------------------------------------ kernel -

constexpr int kChunks = 4;   // 64-entry chunks whose loads phase A issues together

template <typename real, bool ONE, int SCAP, int TI>
__global__ __launch_bounds__(kWave) void k_tersoff(ComputeLaunch a, DeviceTable tab)
{
    __shared__ Shared<real, SCAP> sh;
    const int lane = threadIdx.x;
    const ParamR<real> *ptab = table_r<real>(tab);

    double e_acc = 0.0;
    double w_acc[6] = {0, 0, 0, 0, 0, 0};
    long long n_pairs = 0, n_trip = 0;

    const int B = a.atoms_per_batch;
    const int ngroups = (a.n + B - 1) / B;

    for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        int a0 = grp * B;
        const int a_end = min(a0 + B, a.n);
        while (a0 < a_end) {
            const int nb = a_end - a0;
            // ---- stage centre atoms
            if (lane < nb) {
                const size_t i = (size_t)(a0 + lane);
                double x = a.pos[3 * i], y = a.pos[3 * i + 1], z = a.pos[3 * i + 2];
                sh.xi[lane] = x; sh.yi[lane] = y; sh.zi[lane] = z;
                sh.ti[lane] = ONE ? 0 : a.types[i];
                sh.pcnt[lane] = 0;
                sh.fi[lane][0] = sh.fi[lane][1] = sh.fi[lane][2] = 0.0;
                if (a.pos_build) {
                    double dx = x - a.pos_build[3 * i], dy = y - a.pos_build[3 * i + 1],
                           dz = z - a.pos_build[3 * i + 2];
                    if (!(dx * dx + dy * dy + dz * dz <= a.stale_sq)) atomicOr(a.flags, kFlagStale);
                }
            }
            if (lane < nb) sh.eoff[lane] = a.offsets[a0 + lane];
            if (lane == 0) sh.eoff[nb] = a.offsets[a0 + nb];
            __syncthreads();

            // ---- phase A: skin exclusion and packing.  The index and position
            // loads of up to kChunks 64-entry chunks are issued together so the
            // gathers overlap; chunks are then consumed in order.
            const int e_begin = sh.eoff[0], e_end = sh.eoff[nb];
            int npacked = 0;
            int cut = nb;
            bool stop = false;
            for (int eb = e_begin; eb < e_end && !stop; eb += kWave * kChunks) {
                int jv[kChunks], rv[kChunks], tv[kChunks];
                double xv[kChunks], yv[kChunks], zv[kChunks];
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    const int e = eb + c * kWave + lane;
                    int2 q = e < e_end ? a.jr[e] : make_int2(-1, 0);
                    jv[c] = q.x;
                    rv[c] = q.y;
                }
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    xv[c] = yv[c] = zv[c] = 0.0;
                    tv[c] = 0;
                    if (jv[c] >= 0) {
                        const double *pj = a.pos + 3 * (size_t)jv[c];
                        xv[c] = pj[0]; yv[c] = pj[1]; zv[c] = pj[2];
                        if (!ONE) tv[c] = a.types[jv[c]];
                    }
                }
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    const int e0 = eb + c * kWave;
                    if (stop || e0 >= e_end) break;
                    const int e = e0 + lane;
                    bool acc = false;
                    int al = 0;
                    double dx = 0, dy = 0, dz = 0, rsq = 0;
                    if (e < e_end) {
                        al = find_seg(sh.eoff, nb, e);
                        dx = image(xv[c] - sh.xi[al], a.L[0], a.invL[0]);
                        dy = image(yv[c] - sh.yi[al], a.L[1], a.invL[1]);
                        dz = image(zv[c] - sh.zi[al], a.L[2], a.invL[2]);
                        rsq = norm2(dx, dy, dz);
                        const double psq = ONE ? tab.packsq[0] : tab.packsq[sh.ti[al] * tab.ntypes + tv[c]];
                        acc = rsq < psq;
                    }
                    unsigned long long m = __ballot(acc);
                    const int below = lanes_below(m);
                    const int cnt = __popcll(m);
                    if (npacked + cnt > SCAP) {
                        // cut the batch before the first atom whose slots do not fit
                        unsigned long long over = __ballot(acc && (npacked + below >= SCAP));
                        int fl = __ffsll((long long)over) - 1;
                        cut = __shfl(al, fl, kWave);
                        acc = acc && (al < cut);
                        stop = true;
                    }
                    if (e < e_end && (!stop || al < cut)) a.packed[e] = acc ? 1 : 0;
                    if (acc) {
                        const int s = npacked + below;
                        real r = M<real>::sqrt((real)rsq);
                        real ri = M<real>::rcp(r);
                        sh.rsq[s] = rsq;
                        sh.r[s] = r;
                        sh.rinv[s] = ri;
                        sh.ux[s] = (real)dx * ri;
                        sh.uy[s] = (real)dy * ri;
                        sh.uz[s] = (real)dz * ri;
                        sh.zeta[s] = real(0);
                        sh.j[s] = jv[c];
                        sh.e[s] = rv[c];
                        sh.tj[s] = tv[c];
                        sh.al[s] = al;
                        atomicAdd(&sh.pcnt[al], 1);
                    }
                    if (!stop) npacked += cnt;
                }
            }
            __syncthreads();
            if (cut == 0) {
                // a single atom has more packed neighbours than SCAP: its terms
                // are skipped (reported), none of its entries is marked packed
                if (lane == 0) atomicOr(a.flags, kFlagOverflow);
                for (int e = sh.eoff[0] + lane; e < sh.eoff[1]; e += kWave) {
                    a.packed[e] = 0;
                    double *f = a.contrib + 3 * (size_t)a.jr[e].y;
                    f[0] = f[1] = f[2] = 0.0;
                }
                if (lane == 0) {
                    double *o = a.own + 3 * (size_t)a0;
                    o[0] = o[1] = o[2] = 0.0;
                }
                a0 += 1;
                __syncthreads();
                continue;
            }

            // ---- per-atom slot and triplet offsets
            {
                int p = lane < cut ? sh.pcnt[lane] : 0;
                int t = p * (p - 1);
                int ip = wave_incl_scan(p);
                int it = wave_incl_scan(t);
                if (lane < cut) {
                    sh.pstart[lane + 1] = ip;
                    sh.tstart[lane + 1] = it;
                }
                if (lane == 0) { sh.pstart[0] = 0; sh.tstart[0] = 0; }
                npacked = __shfl(ip, cut - 1, kWave);
            }
            __syncthreads();
            const int ntrip = sh.tstart[cut];
            const bool cached = ntrip <= kWave * TI;

            // ---- phase C: first K loop (zeta and its gradients)
            Trip<real> tc[TI];
            TripIdx tix[TI];
#pragma unroll
            for (int it = 0; it < TI; ++it) {
                const int t = lane + it * kWave;
                tc[it].z = real(0);
                if (t < ntrip) {
                    tix[it] = decode_triplet(sh, cut, t);
                    bool ok = triplet_eval<real, ONE, SCAP>(sh, tix[it], tab, ptab, tc[it], cached);
                    if (ok) {
                        atomicAdd(&sh.zeta[tix[it].sj], tc[it].z);
                        ++n_trip;
                    }
                }
            }
            if (!cached) {
                for (int t = lane + TI * kWave; t < ntrip; t += kWave) {
                    TripIdx ix = decode_triplet(sh, cut, t);
                    Trip<real> o;
                    if (triplet_eval<real, ONE, SCAP>(sh, ix, tab, ptab, o, false)) {
                        atomicAdd(&sh.zeta[ix.sj], o.z);
                        ++n_trip;
                    }
                }
            }
            __syncthreads();

            // ---- phase D: pair terms, bond order, dV/dzeta
            for (int s = lane; s < npacked; s += kWave) {
                const int al = sh.al[s];
                const int ti = ONE ? 0 : sh.ti[al];
                const int tj = ONE ? 0 : sh.tj[s];
                const int nt = ONE ? 1 : tab.ntypes;
                const int e_ij = (ti * nt + tj) * nt + tj;
                const ParamX px = tab.px[e_ij];
                double fsx = 0, fsy = 0, fsz = 0;
                real dz_out = real(0);
                if (ONE || sh.rsq[s] < px.cutsq) {
                    ++n_pairs;
                    const ParamR<real> &q = ptab[e_ij];
                    const real r = sh.r[s];
                    real fc, dfc;
                    cutoff_terms(q, r, fc, dfc);
                    real fr, fa, dfr, dfa;
                    pair_terms(q, r, fr, dfr, fa, dfa);
                    // Eq. (2) in FP64 log form
                    const double zeta = (double)sh.zeta[s];
                    double b = 1.0, db = 0.0;
                    if (zeta > 0.0) {
                        const double x = ::exp(px.eta * (px.logbeta + ::log(zeta)));
                        b = ::exp(-::log1p(x) * px.inv2eta);
                        db = -0.5 * b * x / (zeta * (1.0 + x));
                    }
                    const real br = (real)b;
                    e_acc += 0.5 * (double)fc * ((double)fr + b * (double)fa);
                    const real dvdr = real(0.5) * (dfc * (fr + br * fa) + fc * (dfr + br * dfa));
                    // force on j is -dV/dx_j = -dvdr * u
                    const real fx = -dvdr * sh.ux[s], fy = -dvdr * sh.uy[s], fz = -dvdr * sh.uz[s];
                    fsx = fx; fsy = fy; fsz = fz;
                    atomicAdd(&sh.fi[al][0], -(double)fx);
                    atomicAdd(&sh.fi[al][1], -(double)fy);
                    atomicAdd(&sh.fi[al][2], -(double)fz);
                    const real dxr = r * sh.ux[s], dyr = r * sh.uy[s], dzr = r * sh.uz[s];
                    w_acc[0] += (double)(dxr * fx);
                    w_acc[1] += (double)(dyr * fy);
                    w_acc[2] += (double)(dzr * fz);
                    w_acc[3] += (double)(dxr * fy);
                    w_acc[4] += (double)(dxr * fz);
                    w_acc[5] += (double)(dyr * fz);
                    dz_out = (real)(0.5 * (double)fc * (double)fa * db);
                }
                sh.fs[s][0] = fsx; sh.fs[s][1] = fsy; sh.fs[s][2] = fsz;
                sh.dzeta[s] = dz_out;
            }
            __syncthreads();

            // ---- phase E: second K loop (dV/dzeta times the gradients)
            auto apply = [&](const TripIdx &ix, const Trip<real> &o) {
                const real dzv = sh.dzeta[ix.sj];
                if (dzv == real(0)) return;
                real fj[3], fk[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    fj[c] = -dzv * o.gj[c];
                    fk[c] = -dzv * o.gk[c];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    atomicAdd(&sh.fs[ix.sj][c], (double)fj[c]);
                    atomicAdd(&sh.fs[ix.sk][c], (double)fk[c]);
                    atomicAdd(&sh.fi[ix.al][c], -(double)(fj[c] + fk[c]));
                }
                const real rj = sh.r[ix.sj], rk = sh.r[ix.sk];
                const real dj[3] = {rj * sh.ux[ix.sj], rj * sh.uy[ix.sj], rj * sh.uz[ix.sj]};
                const real dk[3] = {rk * sh.ux[ix.sk], rk * sh.uy[ix.sk], rk * sh.uz[ix.sk]};
                w_acc[0] += (double)(dj[0] * fj[0] + dk[0] * fk[0]);
                w_acc[1] += (double)(dj[1] * fj[1] + dk[1] * fk[1]);
                w_acc[2] += (double)(dj[2] * fj[2] + dk[2] * fk[2]);
                w_acc[3] += (double)(dj[0] * fj[1] + dk[0] * fk[1]);
                w_acc[4] += (double)(dj[0] * fj[2] + dk[0] * fk[2]);
                w_acc[5] += (double)(dj[1] * fj[2] + dk[1] * fk[2]);
            };
            if (cached) {
#pragma unroll
                for (int it = 0; it < TI; ++it) {
                    const int t = lane + it * kWave;
                    if (t < ntrip) apply(tix[it], tc[it]);
                }
            } else {
                for (int t = lane; t < ntrip; t += kWave) {
                    TripIdx ix = decode_triplet(sh, cut, t);
                    Trip<real> o;
                    if (triplet_eval<real, ONE, SCAP>(sh, ix, tab, ptab, o, true)) apply(ix, o);
                }
            }
            __syncthreads();

            // ---- phase F: write this batch's force terms (no atomics): the
            // force on packed neighbour j goes to the entry (j, i) of j's own
            // row, the force on each centre atom to its own slot; the gather
            // kernel adds up each atom's row.
            for (int s = lane; s < npacked; s += kWave) {
                double *f = a.contrib + 3 * (size_t)sh.e[s];
                f[0] = sh.fs[s][0];
                f[1] = sh.fs[s][1];
                f[2] = sh.fs[s][2];
            }
            if (lane < cut) {
                double *o = a.own + 3 * (size_t)(a0 + lane);
                o[0] = sh.fi[lane][0];
                o[1] = sh.fi[lane][1];
                o[2] = sh.fi[lane][2];
            }
            __syncthreads();
            a0 += cut;
        }
    }

    // ---- per-workgroup partial sums of energy, virial and counts
    double v[7] = {e_acc, w_acc[0], w_acc[1], w_acc[2], w_acc[3], w_acc[4], w_acc[5]};
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] = wave_sum(v[c]);
    long long np = n_pairs, ntr = n_trip;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        np += __shfl_xor(np, off, kWave);
        ntr += __shfl_xor(ntr, off, kWave);
    }
    if (lane == 0) {
        double *p = a.partials + 8 * (size_t)blockIdx.x;
#pragma unroll
        for (int c = 0; c < 7; ++c) p[c] = v[c];
        p[7] = 0.0;
        a.counters[2 * (size_t)blockIdx.x] = np;
        a.counters[2 * (size_t)blockIdx.x + 1] = ntr;
    }
}

__global__ void k_finalize(const double *__restrict__ partials, const long long *__restrict__ counters,
                           int grid, double *__restrict__ out, long long *__restrict__ counts)
{
    __shared__ double sh[8][256];
    __shared__ long long shc[2][256];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    long long c0 = 0, c1 = 0;
    for (int b = threadIdx.x; b < grid; b += blockDim.x) {
        for (int c = 0; c < 7; ++c) v[c] += partials[8 * (size_t)b + c];
        c0 += counters[2 * (size_t)b];
        c1 += counters[2 * (size_t)b + 1];
    }
    for (int c = 0; c < 7; ++c) sh[c][threadIdx.x] = v[c];
    shc[0][threadIdx.x] = c0;
    shc[1][threadIdx.x] = c1;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int c = 0; c < 7; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + off];
            shc[0][threadIdx.x] += shc[0][threadIdx.x + off];
            shc[1][threadIdx.x] += shc[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int c = 0; c < 7; ++c) out[c] = sh[c][0];
        counts[0] = shc[0][0];
        counts[1] = shc[1][0];
    }
}

// F_m = (terms of centre m) + sum over the entries (m, i) of m's row that m
// packed of the force centre i's terms put on m.  The packing radius is
// symmetric and r^2 of (m, i) and (i, m) is bit-identical, so m packed i
// exactly when i packed m, and i stored that force at entry (m, i).
// 16 lanes per row, each row read contiguously; lane partial sums reduced
// across the 16 lanes.
__global__ void k_gather_forces(const int *__restrict__ offsets, const unsigned char *__restrict__ packed,
                                const double *__restrict__ contrib, const double *__restrict__ own,
                                int n, double *__restrict__ forces)
{
    const int m = blockIdx.x * (blockDim.x / 16) + threadIdx.x / 16;
    const int l = threadIdx.x % 16;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (m < n) {
        const int e1 = offsets[m + 1];
        for (int e = offsets[m] + l; e < e1; e += 16) {
            if (packed[e]) {
                fx += contrib[3 * (size_t)e];
                fy += contrib[3 * (size_t)e + 1];
                fz += contrib[3 * (size_t)e + 2];
            }
        }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
        fx += __shfl_xor(fx, off, 16);
        fy += __shfl_xor(fy, off, 16);
        fz += __shfl_xor(fz, off, 16);
    }
    if (m < n && l == 0) {
        forces[3 * (size_t)m] = own[3 * (size_t)m] + fx;
        forces[3 * (size_t)m + 1] = own[3 * (size_t)m + 1] + fy;
        forces[3 * (size_t)m + 2] = own[3 * (size_t)m + 2] + fz;
    }
}

__global__ void k_fill_zero(double *p, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = 0.0;
}

constexpr int kScap = 64;
constexpr int kTi = 3;

template <typename real, bool ONE>
int grid_for(int n, int atoms_per_batch)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tersoff<real, ONE, kScap, kTi>,
                                                     kWave, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    long long groups = ((long long)n + atoms_per_batch - 1) / atoms_per_batch;
    long long g = (long long)per_cu * cus;
    if (g > groups) g = groups;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

int compute_grid_size(bool mixed, bool one_type, int n, int atoms_per_batch)
{
    if (mixed) return one_type ? grid_for<float, true>(n, atoms_per_batch) : grid_for<float, false>(n, atoms_per_batch);
    return one_type ? grid_for<double, true>(n, atoms_per_batch) : grid_for<double, false>(n, atoms_per_batch);
}

hipError_t launch_compute(const ComputeLaunch &a, const DeviceTable &t, bool mixed, int grid,
                          hipStream_t s)
{
    const bool one = t.ntypes == 1;
    if (a.atoms_per_batch < 1 || a.atoms_per_batch > kWave) return hipErrorInvalidValue;
    if (mixed) {
        if (one) hipLaunchKernelGGL((k_tersoff<float, true, kScap, kTi>), dim3(grid), dim3(kWave), 0, s, a, t);
        else hipLaunchKernelGGL((k_tersoff<float, false, kScap, kTi>), dim3(grid), dim3(kWave), 0, s, a, t);
    } else {
        if (one) hipLaunchKernelGGL((k_tersoff<double, true, kScap, kTi>), dim3(grid), dim3(kWave), 0, s, a, t);
        else hipLaunchKernelGGL((k_tersoff<double, false, kScap, kTi>), dim3(grid), dim3(kWave), 0, s, a, t);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, const long long *counters, int grid,
                           double *out7, long long *counts_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, partials, counters, grid, out7, counts_out);
    return hipGetLastError();
}

hipError_t launch_gather_forces(const int *offsets, const unsigned char *packed,
                                const double *contrib, const double *own, int n, double *forces,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_forces, dim3((n + 15) / 16), dim3(256), 0, s, offsets, packed,
                       contrib, own, n, forces);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *p, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

}  // namespace tsf
