// Cell-list neighbour build (Section 2: full per-atom list including the
// skin atoms).  Every kernel here evaluates the inclusion predicate with the
// same rounding sequence as its definition:
//   per axis  t = x_j - x_i;  s = rint(t / L);  d = fma(-s, L, t)
//   r^2 = fma(dz, dz, fma(dy, dy, dx * dx));  include j iff r^2 < rcut^2
// with FP contraction disabled, so the lists are bit-identical to any other
// implementation of that predicate.
//
// Steps: bin atoms to cells (count + rank per cell, input checks) ->
// exclusive scan of cell counts -> scatter atom ids and positions into cell
// order -> one wavefront per supercell (a few cells along the last axis)
// tests the atoms of the surrounding cells and writes each of its atoms' rows,
// sorted, to the row buffer (row i at i * cap, cap >= the longest row) ->
// scan of row counts (list length, longest row) -> reverse-entry map.
#include "internal.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace tsf {

namespace {

__device__ inline int cell_index(double x, double L, double w, int nc)
{
    double u = x - L * floor(x / L);
    int c = (int)floor(u / w);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Cell of every atom (positions wrapped into the box for binning only) and
// its rank within the cell; non-finite positions raise flag 1 and types
// outside [0, ntypes) flag 2.
__global__ void k_bin(const double *__restrict__ pos, const int *__restrict__ types, int n, int ntypes,
                      CellGrid g, int *__restrict__ cell_of, int *__restrict__ rank,
                      int *__restrict__ count, int *flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *p = pos + 3 * (size_t)i;
    int f = 0;
    if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) f |= 1;
    const int t = types[i];
    if (t < 0 || t >= ntypes) f |= 2;
    if (f) atomicOr(flags, f);
    int cx = cell_index(p[0], g.L[0], g.cell_w[0], g.nc[0]);
    int cy = cell_index(p[1], g.L[1], g.cell_w[1], g.nc[1]);
    int cz = cell_index(p[2], g.L[2], g.cell_w[2], g.nc[2]);
    int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
    cell_of[i] = c;
    rank[i] = atomicAdd(&count[c], 1);
}

// Cell of every atom of a batch of systems (no input checks: a batch holds
// validated inputs only); cells of system s are numbered from its cell_off.
__global__ void k_bin_systems(const double *__restrict__ pos, const int *__restrict__ sys_of,
                              const SysDesc *__restrict__ sys, const BatchDims *__restrict__ dims,
                              int *__restrict__ cell_of, int *__restrict__ rank, int *__restrict__ count)
{
    const int n = dims->n_atoms;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double *p = pos + 3 * (size_t)i;
        const SysDesc &d = sys[sys_of[i]];
        const CellGrid &g = d.g;
        int cx = cell_index(p[0], g.L[0], g.cell_w[0], g.nc[0]);
        int cy = cell_index(p[1], g.L[1], g.cell_w[1], g.nc[1]);
        int cz = cell_index(p[2], g.L[2], g.cell_w[2], g.nc[2]);
        int c = d.cell_off + (cx * g.nc[1] + cy) * g.nc[2] + cz;
        cell_of[i] = c;
        rank[i] = atomicAdd(&count[c], 1);
    }
}

// n_dev, when not null, holds the atom count (batches); n is then the
// capacity the grid was sized for.
__global__ void k_scatter(const double *__restrict__ pos, int n, const int *__restrict__ n_dev,
                          const int *__restrict__ cell_of, const int *__restrict__ rank,
                          const int *__restrict__ cell_start, int *__restrict__ cell_atoms,
                          double *__restrict__ cell_pos)
{
    const int nn = n_dev ? *n_dev : n;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += gridDim.x * blockDim.x) {
        int slot = cell_start[cell_of[i]] + rank[i];
        cell_atoms[slot] = i;
        cell_pos[3 * (size_t)slot + 0] = pos[3 * (size_t)i + 0];
        cell_pos[3 * (size_t)slot + 1] = pos[3 * (size_t)i + 1];
        cell_pos[3 * (size_t)slot + 2] = pos[3 * (size_t)i + 2];
    }
}

// s = rint(t / L) evaluated as rint(t * (1/L)) whenever that is provably the
// same integer: t * (1/L) is within a few ulps of t / L, so the two round
// alike unless the quotient lies within ~1e-12 (relative) of a half-integer;
// only then is the IEEE division taken.
__device__ inline double image_component(double xj, double xi, double L, double invL)
{
    const double t = xj - xi;
    const double q = t * invL;
    const double fq = q - floor(q);
    double s;
    if (fabs(fq - 0.5) > 1e-12 * fmax(1.0, fabs(q))) s = rint(q);
    else s = rint(t / L);
    return fma(-s, L, t);
}

// Conservative single-precision pre-test: false only if the pair is surely
// outside the list radius.  With t = x_j - x_i in FP64 and u = 2^-24, the
// single-precision minimum image differs from the exact one by at most
// u (2|t| + L + |d|) per axis (or lands on the other image, which for a pair
// within range can only happen when both images lie at L/2 ~ rcs), so
// widening the radius by 2.5e-7 (2 sum|t| + sum L) + 1e-5 never rejects a
// neighbour; survivors get the exact FP64 test.
__device__ inline bool may_be_neighbour(double xj, double yj, double zj, double xi, double yi, double zi,
                                        const CellGrid &g, float rcs)
{
    const float a0 = (float)(xj - xi), a1 = (float)(yj - yi), a2 = (float)(zj - zi);
    const float d0 = fmaf(-rintf(a0 * g.invLf[0]), g.Lf[0], a0);
    const float d1 = fmaf(-rintf(a1 * g.invLf[1]), g.Lf[1], a1);
    const float d2 = fmaf(-rintf(a2 * g.invLf[2]), g.Lf[2], a2);
    const float r2 = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
    const float delta = 2.5e-7f * (2.f * (fabsf(a0) + fabsf(a1) + fabsf(a2)) + g.Lsum) + 1e-5f;
    const float lim = rcs + delta;
    return r2 < lim * lim;
}

// Pre-test on staged single-precision coordinates that already carry the
// periodic image of their stencil cell (relative to the supercell origin):
// for a pair within range that image is the minimum image, so the staged
// difference equals the exact displacement up to a few float roundings of
// coordinates within a few cells of the origin (< 1e-5 A); the radius is
// widened by 1e-4 A.
__device__ inline bool may_be_neighbour_shifted(float xj, float yj, float zj, float xi, float yi, float zi,
                                                float lim2)
{
    const float d0 = xj - xi, d1 = yj - yi, d2 = zj - zi;
    return fmaf(d2, d2, fmaf(d1, d1, d0 * d0)) < lim2;
}

__device__ inline bool in_range(double xj, double yj, double zj, double xi, double yi, double zi,
                                const CellGrid &g, double rc2)
{
    const double dx = image_component(xj, xi, g.L[0], g.invL[0]);
    const double dy = image_component(yj, yi, g.L[1], g.invL[1]);
    const double dz = image_component(zj, zi, g.L[2], g.invL[2]);
    return fma(dz, dz, fma(dy, dy, dx * dx)) < rc2;
}

// One wavefront per supercell: kSuper consecutive cells along the last axis.
// The atoms of the unique cells around it (3 x 3 x (kSuper + 2) cells, or
// fewer on small grids) are staged in LDS.  Fast path: the lanes run over
// all (atom of the supercell, candidate) pairs, a single-precision pre-test
// keeps the possible neighbours, the exact FP64 predicate decides them, the
// accepted pairs are packed in order (ballot + prefix count), and every row
// is rank-sorted by j and written to the fixed-capacity row buffer.
// Supercells with too many candidates or pairs take the general path: one
// atom at a time, candidates in chunks.
constexpr int kSuper = 4;
constexpr int kCandCap = 256;
constexpr int kRowCap = kMaxRow;
constexpr int kSurvCap = 512;
constexpr int kCellAtomCap = 64;
constexpr int kMaxStencil = 3 * 3 * (kSuper + 2);

struct SearchLDS {
    int cj[kCandCap];
    double cx[kCandCap], cy[kCandCap], cz[kCandCap];
    float fx[kCandCap], fy[kCandCap], fz[kCandCap];
    int row[kRowCap];
    int surv[kSurvCap];
    int pa[kSurvCap], pj[kSurvCap];
    int rowcnt[kCellAtomCap], rowst[kCellAtomCap];
    int pre[kMaxStencil + 1], st[kMaxStencil];
    double shx[kMaxStencil], shy[kMaxStencil], shz[kMaxStencil];
};

// Rows of the atoms of supercell sc of grid g, whose cells are numbered from
// cell_off.  A row longer than cap is not written; its row_count is the true
// length (CLAMP false) or 0 with bit 1 raised in *sys_flags (CLAMP true, for
// batches whose kernels run without a host check in between).
template <bool CLAMP>
__device__ __forceinline__ void search_supercell(SearchLDS &sm, const CellGrid &g, int cell_off, int sc,
                                                 double rc2, const int *__restrict__ cell_start,
                                                 const int *__restrict__ cell_count,
                                                 const int *__restrict__ cell_atoms,
                                                 const double *__restrict__ cpos, int cap,
                                                 int *__restrict__ ell, int *__restrict__ row_count,
                                                 int *sys_flags)
{
    const int lane = threadIdx.x;
    const int nsz = (g.nc[2] + kSuper - 1) / kSuper;          // supercells per column
    const int n0 = g.nc[0] >= 3 ? 3 : g.nc[0];
    const int n1 = g.nc[1] >= 3 ? 3 : g.nc[1];
    const bool zall = g.nc[2] < kSuper + 2;                    // small grid: every z cell once
    const int n2 = zall ? g.nc[2] : kSuper + 2;
    const int nq = n0 * n1 * n2;
    const float rcs = (float)sqrt(rc2);
    // the stencil fixes each candidate's periodic image when every axis has
    // at least three cells around the supercell
    const bool shifted = n0 == 3 && n1 == 3 && !zall;
    const float lim = rcs + 1e-4f, lim2 = lim * lim;
    auto store_count = [&](int i, int cnt) {
        if (CLAMP && cnt > cap) {
            row_count[i] = 0;
            atomicOr(sys_flags, 1);
        } else {
            row_count[i] = cnt;
        }
    };

    const int col = sc / nsz;                              // (x, y) column
    const int z0 = (sc - col * nsz) * kSuper;
    const int kz = min(kSuper, g.nc[2] - z0);
    const int cx0 = col / g.nc[1], cy0 = col % g.nc[1];
    const int c_first = cell_off + (cx0 * g.nc[1] + cy0) * g.nc[2] + z0;
    // stencil cells: x, y offsets {-1,0,1} (or all cells when nc < 3), z from z0-1 to z0+kSuper
    int cntq = 0, stq = 0;
    if (lane < nq) {
        const int q0 = lane / (n1 * n2), q1 = (lane / n2) % n1, q2 = lane % n2;
        int x = cx0 + (n0 == 3 ? q0 - 1 : q0 - cx0);
        int y = cy0 + (n1 == 3 ? q1 - 1 : q1 - cy0);
        int z = zall ? q2 : z0 - 1 + q2;
        double sx = 0, sy = 0, sz = 0;   // image shift of this stencil cell
        if (x < 0) { x += g.nc[0]; sx = -g.L[0]; } else if (x >= g.nc[0]) { x -= g.nc[0]; sx = g.L[0]; }
        if (y < 0) { y += g.nc[1]; sy = -g.L[1]; } else if (y >= g.nc[1]) { y -= g.nc[1]; sy = g.L[1]; }
        if (z < 0) { z += g.nc[2]; sz = -g.L[2]; } else if (z >= g.nc[2]) { z -= g.nc[2]; sz = g.L[2]; }
        const int cc = cell_off + (x * g.nc[1] + y) * g.nc[2] + z;
        stq = cell_start[cc];
        cntq = cell_count[cc];
        sm.shx[lane] = sx; sm.shy[lane] = sy; sm.shz[lane] = sz;
    }
    const int cs = cell_start[c_first];
    const int A = cell_start[c_first + kz - 1] + cell_count[c_first + kz - 1] - cs;
    int incl = cntq;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(incl, off, 64);
        if (lane >= off) incl += u;
    }
    if (A == 0) return;
    const int T = __shfl(incl, nq - 1, 64);
    if (lane < nq) {
        sm.pre[lane] = incl - cntq;
        sm.st[lane] = stq;
    }
    if (lane == 0) sm.pre[nq] = T;
    __syncthreads();
    const double ox = cx0 * g.cell_w[0], oy = cy0 * g.cell_w[1], oz = z0 * g.cell_w[2];
    // staged position of the supercell's first atom: stencil cell (centre x, centre y, z0)
    const int qf = (n0 == 3 ? 1 : cx0) * n1 * n2 + (n1 == 3 ? 1 : cy0) * n2 + (zall ? z0 : 1);
    auto stage = [&](int t0, int tn) {
        for (int tt = lane; tt < tn; tt += 64) {
            const int t = t0 + tt;
            int lo = 0, hi = nq - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (sm.pre[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int sidx = sm.st[lo] + (t - sm.pre[lo]);
            sm.cj[tt] = cell_atoms[sidx];
            const double x = cpos[3 * (size_t)sidx], y = cpos[3 * (size_t)sidx + 1], z = cpos[3 * (size_t)sidx + 2];
            sm.cx[tt] = x; sm.cy[tt] = y; sm.cz[tt] = z;
            if (shifted) {
                // wrapped coordinate as in the binning, plus the cell's image shift
                sm.fx[tt] = (float)(x - g.L[0] * floor(x / g.L[0]) + sm.shx[lo] - ox);
                sm.fy[tt] = (float)(y - g.L[1] * floor(y / g.L[1]) + sm.shy[lo] - oy);
                sm.fz[tt] = (float)(z - g.L[2] * floor(z / g.L[2]) + sm.shz[lo] - oz);
            }
        }
    };
    const bool one_chunk = T <= kCandCap;
    if (one_chunk) stage(0, T);
    __syncthreads();

    bool fast = one_chunk && A <= kCellAtomCap;
    int nsurv = 0;
    const unsigned magic = 0xFFFFFFFFu / (unsigned)max(T, 1) + 1u;   // f / T = umulhi(f, magic), f, T < 2^16
    const int ic0 = sm.pre[qf];
    if (fast) {
        // pass 1: single-precision pre-test over all (atom, candidate) pairs
        const int AT = A * T;
        for (int base = 0; base < AT; base += 64) {
            const int f = base + lane;
            bool keep = false;
            if (f < AT) {
                const int ia = (int)__umulhi((unsigned)f, magic);
                const int t = f - ia * T;
                const int ti = ic0 + ia;
                if (t != ti)
                    keep = shifted ? may_be_neighbour_shifted(sm.fx[t], sm.fy[t], sm.fz[t], sm.fx[ti], sm.fy[ti],
                                                              sm.fz[ti], lim2)
                                   : may_be_neighbour(sm.cx[t], sm.cy[t], sm.cz[t], sm.cx[ti], sm.cy[ti],
                                                      sm.cz[ti], g, rcs);
            }
            const unsigned long long m = __ballot(keep);
            const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            if (keep && nsurv + below < kSurvCap) sm.surv[nsurv + below] = f;
            nsurv += __popcll(m);
        }
        fast = nsurv <= kSurvCap;
    }
    if (fast) {
        __syncthreads();
        // pass 2: exact predicate on the survivors, accepted pairs kept in order
        int nacc = 0;
        for (int base = 0; base < nsurv; base += 64) {
            const int k = base + lane;
            bool acc = false;
            int ia = 0, t = 0;
            if (k < nsurv) {
                const int f = sm.surv[k];
                ia = (int)__umulhi((unsigned)f, magic);
                t = f - ia * T;
                const int ti = ic0 + ia;
                acc = in_range(sm.cx[t], sm.cy[t], sm.cz[t], sm.cx[ti], sm.cy[ti], sm.cz[ti], g, rc2);
            }
            const unsigned long long m = __ballot(acc);
            const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            if (acc) {
                sm.pa[nacc + below] = ia;
                sm.pj[nacc + below] = sm.cj[t];
            }
            nacc += __popcll(m);
        }
        if (lane < A) sm.rowcnt[lane] = 0;
        __syncthreads();
        for (int k = lane; k < nacc; k += 64) atomicAdd(&sm.rowcnt[sm.pa[k]], 1);
        __syncthreads();
        {
            const int v = lane < A ? sm.rowcnt[lane] : 0;
            int inc = v;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                int u = __shfl_up(inc, off, 64);
                if (lane >= off) inc += u;
            }
            if (lane < A) sm.rowst[lane] = inc - v;
        }
        __syncthreads();
        for (int k = lane; k < nacc; k += 64) {
            const int ia = sm.pa[k], v = sm.pj[k];
            const int r0 = sm.rowst[ia], rn = sm.rowcnt[ia];
            if (rn <= cap) {
                int rk = 0;
                for (int q = 0; q < rn; ++q) rk += sm.pj[r0 + q] < v;
                ell[(size_t)sm.cj[ic0 + ia] * cap + rk] = v;
            }
        }
        if (lane < A) store_count(sm.cj[ic0 + lane], sm.rowcnt[lane]);
        __syncthreads();
        return;
    }

    // general path: one atom at a time, candidates in chunks
    for (int ia = 0; ia < A; ++ia) {
        const int si = cs + ia;
        const int i = cell_atoms[si];
        const double xi = cpos[3 * (size_t)si], yi = cpos[3 * (size_t)si + 1], zi = cpos[3 * (size_t)si + 2];
        int cnt = 0;
        for (int t0 = 0; t0 < T; t0 += kCandCap) {
            const int tn = min(kCandCap, T - t0);
            if (!one_chunk) {
                __syncthreads();
                stage(t0, tn);
                __syncthreads();
            }
            for (int tb = 0; tb < tn; tb += 64) {
                const int tt = tb + lane;
                bool acc = false;
                int j = 0;
                if (tt < tn) {
                    j = sm.cj[tt];
                    if (j != i) acc = in_range(sm.cx[tt], sm.cy[tt], sm.cz[tt], xi, yi, zi, g, rc2);
                }
                const unsigned long long m = __ballot(acc);
                const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                if (acc && cnt + below < kRowCap) sm.row[cnt + below] = j;
                cnt += __popcll(m);
            }
        }
        __syncthreads();
        if (cnt <= cap && cnt <= kRowCap) {
            int *out = ell + (size_t)i * cap;
            for (int e = lane; e < cnt; e += 64) {
                const int v = sm.row[e];
                int rk = 0;
                for (int q = 0; q < cnt; ++q) rk += sm.row[q] < v;
                out[rk] = v;
            }
        }
        if (lane == 0) store_count(i, cnt);
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_search_cells(CellGrid g, double rc2, const int *__restrict__ cell_start,
                                                     const int *__restrict__ cell_count,
                                                     const int *__restrict__ cell_atoms,
                                                     const double *__restrict__ cpos, int nsuper, int cap,
                                                     int *__restrict__ ell, int *__restrict__ row_count)
{
    __shared__ SearchLDS sm;
    for (int sc = blockIdx.x; sc < nsuper; sc += gridDim.x)
        search_supercell<false>(sm, g, 0, sc, rc2, cell_start, cell_count, cell_atoms, cpos, cap, ell,
                                row_count, nullptr);
}

// Batched form: the supercells of every system of the batch, numbered from
// each system's super_off; the system of a supercell is found by bisection.
__global__ __launch_bounds__(64) void k_search_systems(const SysDesc *__restrict__ sys,
                                                       const BatchDims *__restrict__ dims, double rc2,
                                                       const int *__restrict__ cell_start,
                                                       const int *__restrict__ cell_count,
                                                       const int *__restrict__ cell_atoms,
                                                       const double *__restrict__ cpos, int cap,
                                                       int *__restrict__ ell, int *__restrict__ row_count,
                                                       int *__restrict__ sys_status)
{
    __shared__ SearchLDS sm;
    const int nsuper = dims->n_super, nsys = dims->n_sys;
    for (int sc = blockIdx.x; sc < nsuper; sc += gridDim.x) {
        int lo = 0, hi = nsys - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sys[mid].super_off <= sc) lo = mid; else hi = mid - 1;
        }
        const CellGrid g = sys[lo].g;
        search_supercell<true>(sm, g, sys[lo].cell_off, sc - sys[lo].super_off, rc2, cell_start, cell_count,
                               cell_atoms, cpos, cap, ell, row_count, sys_status + lo);
    }
}

// rv[e] for entry e = (i, j) = i * cap + q of the row buffer: the entry of i
// in the sorted row of j.  One thread per (i, q) with i < j searches row j
// (16-entry pieces of four 16-byte loads issued together) and fills both
// rv[(i, j)] and rv[(j, i)].  The inclusion predicate is symmetric (negating
// t negates s and d exactly), so the entry exists; a missing one raises
// flag 4.
__device__ __forceinline__ void reverse_entry(const int *__restrict__ ell, int cap,
                                              const int *__restrict__ row_count, unsigned tid,
                                              int *__restrict__ rv, int *flags)
{
    const int i = (int)(tid / (unsigned)cap);
    const int q = (int)(tid - (unsigned)i * (unsigned)cap);
    if (q >= row_count[i]) return;
    const int j = ell[(size_t)i * cap + q];
    if (j < i) return;   // the pair is handled from the other side
    const int cj = row_count[j];
    const int4 *row = reinterpret_cast<const int4 *>(ell + (size_t)j * cap);
    int at = -1;
    for (int b = 0; b < cj && at < 0; b += 16) {
        int4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (b + 4 * u < cap) ? row[(b >> 2) + u] : make_int4(-1, -1, -1, -1);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = b + 4 * u;
            if (k + 0 < cj && v[u].x == i) at = k + 0;
            if (k + 1 < cj && v[u].y == i) at = k + 1;
            if (k + 2 < cj && v[u].z == i) at = k + 2;
            if (k + 3 < cj && v[u].w == i) at = k + 3;
        }
    }
    const int e = (int)((size_t)i * cap + q);
    if (at < 0) {
        atomicOr(flags, 4);
        rv[e] = e;
    } else {
        const int f = (int)((size_t)j * cap + at);
        rv[e] = f;
        rv[f] = e;
    }
}

// One thread per (i, q), q < cap; n_dev as in k_scatter.
__global__ void k_reverse_map(const int *__restrict__ ell, int cap, const int *__restrict__ row_count, int n,
                              const int *__restrict__ n_dev, int *__restrict__ rv, int *flags)
{
    const unsigned total = (unsigned)(n_dev ? *n_dev : n) * (unsigned)cap;   // n * cap < 2^31
    for (unsigned tid = blockIdx.x * blockDim.x + threadIdx.x; tid < total; tid += gridDim.x * blockDim.x)
        reverse_entry(ell, cap, row_count, tid, rv, flags);
}

// ---- exclusive scan (three passes) -----------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 4;
constexpr int kScanTile = kScanThreads * kScanPerThread;

__device__ inline int block_excl_scan(int v, int *sh, int &total)
{
    // Hillis-Steele over 256 threads in shared memory
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int incl = sh[t];
    total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tiles(const int *__restrict__ in, int *__restrict__ out, int n,
                             int *__restrict__ tile_sum, int *__restrict__ tile_max)
{
    __shared__ int sh[kScanThreads];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanPerThread;
    int v[kScanPerThread];
    int s = 0, mx = 0;
    for (int q = 0; q < kScanPerThread; ++q) {
        v[q] = (base + q < n) ? in[base + q] : 0;
        s += v[q];
        mx = v[q] > mx ? v[q] : mx;
    }
    int total;
    int ex = block_excl_scan(s, sh, total);
    for (int q = 0; q < kScanPerThread; ++q) {
        if (base + q < n) out[base + q] = ex;
        ex += v[q];
    }
    // block max
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tile_sum[blockIdx.x] = total;
        tile_max[blockIdx.x] = sh[0];
    }
}

// One block scans the tile sums (exclusive, in place) in chunks of 256 with
// a running carry; writes the grand total to out[n] and the max to *max_out.
__global__ void k_scan_tile_sums(int *__restrict__ tile_sum, const int *__restrict__ tile_max,
                                 int ntiles, int *__restrict__ out, int n, int *max_out)
{
    __shared__ int sh[kScanThreads];
    int carry = 0, mx = 0;
    for (int c0 = 0; c0 < ntiles; c0 += kScanThreads) {
        int t = c0 + threadIdx.x;
        int v = t < ntiles ? tile_sum[t] : 0;
        int m = t < ntiles ? tile_max[t] : 0;
        mx = m > mx ? m : mx;
        int total;
        int ex = block_excl_scan(v, sh, total);
        if (t < ntiles) tile_sum[t] = ex + carry;
        carry += total;
    }
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[n] = carry;
        if (max_out) *max_out = sh[0];
    }
}

__global__ void k_scan_add(int *__restrict__ out, int n, const int *__restrict__ tile_sum)
{
    int base = blockIdx.x * kScanTile;
    int add = tile_sum[blockIdx.x];
    for (int q = threadIdx.x; q < kScanTile; q += kScanThreads)
        if (base + q < n) out[base + q] += add;
}

inline int blocks_for(long long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

size_t scan_tmp_size(int n)
{
    return 2 * (size_t)blocks_for(n > 0 ? n : 1, kScanTile);
}

hipError_t launch_exclusive_scan(const int *in, int *out, int n, int *tmp, int *max_out,
                                 hipStream_t s)
{
    int ntiles = blocks_for(n > 0 ? n : 1, kScanTile);
    int *tile_sum = tmp, *tile_max = tmp + ntiles;
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kScanThreads), 0, s, in, out, n,
                       tile_sum, tile_max);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kScanThreads), 0, s, tile_sum, tile_max,
                       ntiles, out, n, max_out);
    hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(kScanThreads), 0, s, out, n, tile_sum);
    return hipGetLastError();
}

hipError_t launch_reverse_map(const int *ell, int cap, const int *row_count, int n, const int *n_dev, int *rv,
                              int *flags, hipStream_t s)
{
    const long long threads = (long long)n * cap;
    long long blocks = (threads + 255) / 256;
    if (n_dev && blocks > kBatchGrid) blocks = kBatchGrid;
    hipLaunchKernelGGL(k_reverse_map, dim3((unsigned)std::max(1LL, blocks)), dim3(256), 0, s, ell, cap,
                       row_count, n, n_dev, rv, flags);
    return hipGetLastError();
}

hipError_t launch_bin_atoms(const double *pos, const int *types, int n, int ntypes, const CellGrid &g,
                            int *cell_of, int *rank_in_cell, int *cell_count, int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos, types, n, ntypes, g, cell_of,
                       rank_in_cell, cell_count, flags);
    return hipGetLastError();
}

hipError_t launch_bin_systems(const double *pos, const int *sys_of, const SysDesc *sys, const BatchDims *dims,
                              int max_atoms, int *cell_of, int *rank_in_cell, int *cell_count, hipStream_t s)
{
    const int grid = std::max(1, std::min(blocks_for(max_atoms, 256), kBatchGrid));
    hipLaunchKernelGGL(k_bin_systems, dim3(grid), dim3(256), 0, s, pos, sys_of, sys, dims, cell_of, rank_in_cell,
                       cell_count);
    return hipGetLastError();
}

hipError_t launch_scatter_cells(const double *pos, int n, const int *n_dev, const int *cell_of,
                                const int *rank_in_cell, const int *cell_start,
                                int *cell_atoms, double *cell_pos, hipStream_t s)
{
    int grid = blocks_for(n, 256);
    if (n_dev) grid = std::min(grid, kBatchGrid);
    hipLaunchKernelGGL(k_scatter, dim3(std::max(1, grid)), dim3(256), 0, s, pos, n, n_dev, cell_of,
                       rank_in_cell, cell_start, cell_atoms, cell_pos);
    return hipGetLastError();
}

namespace {
int search_grid(const void *kern, int nsuper)
{
    int per_cu = 0, dev = 0, cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return std::max(1, std::min(nsuper, per_cu * cus));
}
}  // namespace

hipError_t launch_search_systems(const SysDesc *sys, const BatchDims *dims, int max_super, double rcut,
                                 const int *cell_start, const int *cell_count, const int *cell_atoms,
                                 const double *cell_pos, int cap, int *ell, int *row_count, int *sys_status,
                                 hipStream_t s)
{
    const int grid = search_grid((const void *)k_search_systems, max_super);
    hipLaunchKernelGGL(k_search_systems, dim3(grid), dim3(64), 0, s, sys, dims, rcut * rcut, cell_start,
                       cell_count, cell_atoms, cell_pos, cap, ell, row_count, sys_status);
    return hipGetLastError();
}

hipError_t launch_search(const CellGrid &g, double rcut, const int *cell_start, const int *cell_count,
                         const int *cell_atoms, const double *cell_pos, int ncell, int cap, int *ell,
                         int *row_count, hipStream_t s)
{
    (void)ncell;
    const int nsuper = g.nc[0] * g.nc[1] * ((g.nc[2] + kSuper - 1) / kSuper);
    const int grid = search_grid((const void *)k_search_cells, nsuper);
    hipLaunchKernelGGL(k_search_cells, dim3(grid), dim3(64), 0, s, g, rcut * rcut, cell_start, cell_count,
                       cell_atoms, cell_pos, nsuper, cap, ell, row_count);
    return hipGetLastError();
}

int supercells(const int nc[3]) { return nc[0] * nc[1] * ((nc[2] + kSuper - 1) / kSuper); }

}  // namespace tsf
