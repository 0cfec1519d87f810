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
// order -> one thread per atom tests the atoms of the 27 surrounding cells and
// writes its row, sorted, to the row buffer (row i at i * cap, cap >= the
// longest row; rows too long for the thread's LDS buffer go to a wavefront
// per row) -> scan of row counts (list length, longest row) -> compaction of
// the rows into the list.
#include "internal.h"

#include <algorithm>
#include <climits>
#include <type_traits>

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
// outside [0, ntypes) flag 2.  The types are copied to types_out.  Also adds
// into *near_count the consecutive atoms (i, i + 1) of one wavefront (i not
// the last atom of a 64-atom group) whose cells are the same or adjacent
// (periodically) along every axis: how coherent in space the caller's atom
// order is.  Blocks of kBinThreads threads.
constexpr int kBinThreads = 256;
__global__ __launch_bounds__(kBinThreads) void k_bin(const double *__restrict__ pos, const int *__restrict__ types,
                                                     int n, int ntypes, CellGrid g, int *__restrict__ cell_of,
                                                     int *__restrict__ rank, int *__restrict__ count, int *flags,
                                                     int *__restrict__ types_out, int *__restrict__ near_count)
{
    __shared__ int part[kBinThreads / kWave];
    auto near = [](int u, int v, int m) {
        const int d = u > v ? u - v : v - u;
        return d <= 1 || d == m - 1;
    };
    const int lane = threadIdx.x % kWave;
    int nc = 0;   // this thread's near pairs
    const ItemRange r = xcd_items((n + blockDim.x - 1) / blockDim.x);
    for (int it = r.begin; it < r.end; it += r.stride) {   // the same trip count in every lane of a block
        const int i = it * blockDim.x + threadIdx.x;
        const bool valid = i < n;
        int cx = 0, cy = 0, cz = 0;
        if (valid) {
            const double *p = pos + 3 * (size_t)i;
            int f = 0;
            if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) f |= 1;
            const int t = types[i];
            types_out[i] = t;
            if (t < 0 || t >= ntypes) f |= 2;
            if (f) atomicOr(flags, f);
            cx = cell_index(p[0], g.L[0], g.cell_w[0], g.nc[0]);
            cy = cell_index(p[1], g.L[1], g.cell_w[1], g.nc[1]);
            cz = cell_index(p[2], g.L[2], g.cell_w[2], g.nc[2]);
            const int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
            cell_of[i] = c;
            rank[i] = atomicAdd(&count[c], 1);
        }
        // the cell of atom i + 1: the next lane's
        const int nx = __shfl_down(cx, 1, kWave), ny = __shfl_down(cy, 1, kWave), nz = __shfl_down(cz, 1, kWave);
        if (valid && i + 1 < n && lane != kWave - 1)
            nc += near(cx, nx, g.nc[0]) && near(cy, ny, g.nc[1]) && near(cz, nz, g.nc[2]) ? 1 : 0;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) nc += __shfl_xor(nc, off, kWave);
    if (lane == 0) part[threadIdx.x / kWave] = nc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBinThreads / kWave; ++w) t += part[w];
        if (t) atomicAdd(near_count, t);
    }
}

// Cell of every atom of a batch of systems (no input checks: a batch holds
// validated inputs only); cells of system s are numbered from its cell_off.
__global__ void k_bin_systems(const double *__restrict__ pos, const int *__restrict__ sys_of,
                              const SysDesc *__restrict__ sys, const BatchDims *__restrict__ dims,
                              int *__restrict__ cell_of, int *__restrict__ rank, int *__restrict__ count)
{
    const int n = dims->n_atoms;
    const ItemRange r = xcd_items((n + blockDim.x - 1) / blockDim.x);
    for (int it = r.begin; it < r.end; it += r.stride) {
        const int i = it * blockDim.x + threadIdx.x;
        if (i >= n) continue;
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

// Atom ids and positions in cell order; also the position wrapped into the
// box (as in the binning) in single precision, with the atom id in the fourth
// word, for the search's pre-test.  BATCHED: each atom's box is its system's.
template <bool BATCHED>
__global__ void k_scatter(ScatterLaunch a)
{
    const int nn = BATCHED ? a.dims->n_atoms : a.n;
    const ItemRange r = xcd_items((nn + blockDim.x - 1) / blockDim.x);
    for (int it = r.begin; it < r.end; it += r.stride) {
        const int i = it * blockDim.x + threadIdx.x;
        if (i >= nn) continue;
        const int ci = a.cell_of[i];
        const int slot = a.cell_start[ci] + a.rank[i];
        a.slot_cell[slot] = ci;
        const double x = a.pos[3 * (size_t)i + 0], y = a.pos[3 * (size_t)i + 1], z = a.pos[3 * (size_t)i + 2];
        const CellGrid &g = BATCHED ? a.sys[a.sys_of[i]].g : a.g;
        a.cell_atoms[slot] = i;
        if (a.pos_copy) {
            a.pos_copy[3 * (size_t)i + 0] = x;
            a.pos_copy[3 * (size_t)i + 1] = y;
            a.pos_copy[3 * (size_t)i + 2] = z;
        }
        a.cell_pos[3 * (size_t)slot + 0] = x;
        a.cell_pos[3 * (size_t)slot + 1] = y;
        a.cell_pos[3 * (size_t)slot + 2] = z;
        float4 f;
        f.x = (float)(x - g.L[0] * floor(x / g.L[0]));
        f.y = (float)(y - g.L[1] * floor(y / g.L[1]));
        f.z = (float)(z - g.L[2] * floor(z / g.L[2]));
        f.w = __int_as_float(i);
        a.cell_posf[slot] = f;
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

__device__ inline bool in_range(double xj, double yj, double zj, double xi, double yi, double zi,
                                const CellGrid &g, double rc2)
{
    const double dx = image_component(xj, xi, g.L[0], g.invL[0]);
    const double dy = image_component(yj, yi, g.L[1], g.invL[1]);
    const double dz = image_component(zj, zi, g.L[2], g.invL[2]);
    return fma(dz, dz, fma(dy, dy, dx * dx)) < rc2;
}

// One thread per atom, atoms taken in cell order (neighbouring threads share
// most stencil cells, so candidate data come from cache), in three phases
// whose bodies do not diverge much across the wavefront:
//   1  walk the 27 cells around the atom's own (every cell once along an axis
//      with fewer than three cells) and keep the candidates that pass a
//      single-precision pre-test on the wrapped coordinates -- with the
//      stencil cell's periodic image added when every axis has at least three
//      cells, else by a single-precision minimum image -- in the thread's
//      column of an LDS buffer;
//   2  decide the survivors with the exact FP64 predicate, compacting the
//      accepted neighbour ids in place;
//   3  sort the row with a 32-element bitonic network in registers.
// Atoms with more than kLBuf - 1 survivors are listed for k_search_long.
//
// Pre-test bound: the wrapped single-precision coordinates and the rounded box
// lengths are each within 2^-24 L of their exact values; the shift form
// rounds the image-shifted centre (at most 2^-23 L: it lies in (-L, 2L))
// and the minimum-image form the difference and its correction (at most
// 2^-24 L each); the last difference of an in-range pair rounds by at most
// 2^-24 (rc + delta), so every component is within 6 * 2^-24 L_a (plus that)
// of the exact minimum-image displacement, and the
// single-precision distance within delta = 4e-7 (Lx + Ly + Lz) + 1e-5 of the
// exact one (the 1e-5 covers the rounding of r^2 and of the radius).  So no
// neighbour is rejected by the test r < rc + delta, and, in the shift form, a
// candidate with r < rc - delta is inside for the exact predicate too; only
// the survivors in between take the FP64 test.  (The minimum-image form can
// pick the other image for a pair at almost exactly half a box, so there
// every survivor takes the FP64 test.)
constexpr int kLRow = 32;          // width of the register sort
constexpr int kLBuf = 24;          // LDS slots per thread: up to kLBuf - 1 survivors, one scratch slot
                                   // (24 KB per workgroup: six workgroups per CU)
static_assert(kLBuf <= kLRow, "a row fits the sort");
constexpr int kSearchThreads = 256;

struct StencilCell {
    int cell;          // cell index (with the system's offset)
    float sx, sy, sz;  // periodic image shift of the cell's atoms
};

// Stencil cell q (0 <= q < n0 n1 n2) around local cell (cx, cy, cz).
__device__ __forceinline__ StencilCell stencil_cell(const CellGrid &g, int coff, int cx, int cy, int cz, int n0,
                                                    int n1, int n2, int q)
{
    const int q0 = q / (n1 * n2), q1 = (q / n2) % n1, q2 = q % n2;
    int x = n0 == 3 ? cx + q0 - 1 : q0;
    int y = n1 == 3 ? cy + q1 - 1 : q1;
    int z = n2 == 3 ? cz + q2 - 1 : q2;
    StencilCell c;
    c.sx = c.sy = c.sz = 0.f;
    if (x < 0) { x += g.nc[0]; c.sx = -g.Lf[0]; } else if (x >= g.nc[0]) { x -= g.nc[0]; c.sx = g.Lf[0]; }
    if (y < 0) { y += g.nc[1]; c.sy = -g.Lf[1]; } else if (y >= g.nc[1]) { y -= g.nc[1]; c.sy = g.Lf[1]; }
    if (z < 0) { z += g.nc[2]; c.sz = -g.Lf[2]; } else if (z >= g.nc[2]) { z -= g.nc[2]; c.sz = g.Lf[2]; }
    c.cell = coff + (x * g.nc[1] + y) * g.nc[2] + z;
    return c;
}

// Ascending bitonic sort of 32 values held in registers (constant indices
// only, so the array never leaves registers).
__device__ __forceinline__ void bitonic32(int (&v)[kLRow])
{
#pragma unroll
    for (int k = 2; k <= kLRow; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < kLRow; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const int lo = min(v[i], v[l]), hi = max(v[i], v[l]);
                    if ((i & k) == 0) { v[i] = lo; v[l] = hi; }
                    else { v[i] = hi; v[l] = lo; }
                }
            }
        }
    }
}

template <bool BATCHED>
__global__ __launch_bounds__(kSearchThreads) void k_search_atoms(SearchLaunch a)
{
    __shared__ int buf[kLBuf][kSearchThreads];
    const int tl = threadIdx.x;
    const int n = BATCHED ? a.dims->n_atoms : a.n;
    const ItemRange items = xcd_items((n + kSearchThreads - 1) / kSearchThreads);
    // the atom of cell-order slot t and its cell, loaded one iteration ahead
    float4 fi_next = make_float4(0.f, 0.f, 0.f, 0.f);
    int cell_next = 0;
    auto fetch = [&](int it2) {
        const int t2 = it2 * kSearchThreads + tl;
        if (it2 < items.end && t2 < n) {
            fi_next = a.cell_posf[t2];
            cell_next = a.slot_cell[t2];
        }
    };
    fetch(items.begin);
    for (int it = items.begin; it < items.end; it += items.stride) {
        const int t = it * kSearchThreads + tl;
        const float4 fi = fi_next;
        const int cell_t = cell_next;
        fetch(it + items.stride);
        if (t >= n) continue;
        const int i = __float_as_int(fi.w);
        int coff = 0;
        int *sys_flags = nullptr;
        CellGrid g;
        if constexpr (BATCHED) {
            const int sidx = a.sys_of[i];
            g = a.sys[sidx].g;
            coff = a.sys[sidx].cell_off;
            sys_flags = a.sys_status + sidx;
        } else {
            g = a.g;
        }
        const int c = cell_t - coff;
        const int cz = c % g.nc[2], cy = (c / g.nc[2]) % g.nc[1], cx = c / (g.nc[1] * g.nc[2]);
        const int n0 = min(g.nc[0], 3), n1 = min(g.nc[1], 3), n2 = min(g.nc[2], 3);
        const bool shifted = n0 == 3 && n1 == 3 && n2 == 3;
        const float delta = 4e-7f * (g.Lf[0] + g.Lf[1] + g.Lf[2]) + 1e-5f;
        const float lim = a.rcs + delta, lim2 = lim * lim;
        // below this radius the exact predicate is certain to accept (shift form only)
        const float sure = fmaxf(a.rcs - delta, 0.f), sure2 = sure * sure;

        // ---- 1: pre-test, survivors (candidate slots) to LDS.  The cells
        // (x, y, z-1 .. z+1) of a column are consecutive in cell order, so
        // their atoms form one contiguous range unless the column wraps.
        int ns = 0;
        // SH: add the stencil image shift (every axis has at least three
        // cells) or take the single-precision minimum image
        // ZS: the range carries a z image shift.  The loads of a group of four
        // may run up to three entries past the range (the array is padded by
        // kPosPad entries); those candidates fail u < u1.
        auto scan = [&](auto sh_tag, auto zs_tag, int u0, int u1, float sx, float sy, float sz) {
            constexpr bool SH = decltype(sh_tag)::value;
            constexpr bool ZS = decltype(zs_tag)::value;
            // the centre with the stencil cell's image shift taken off
            const float ox = fi.x - sx, oy = fi.y - sy, oz = ZS ? fi.z - sz : fi.z;
            for (int ub = u0; ub < u1; ub += 4) {
                float4 fj[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) fj[r] = a.cell_posf[ub + r];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int u = ub + r;
                    float d0, d1, d2;
                    if constexpr (SH) {
                        d0 = fj[r].x - ox;
                        d1 = fj[r].y - oy;
                        d2 = fj[r].z - oz;
                    } else {
                        d0 = fj[r].x - fi.x;
                        d1 = fj[r].y - fi.y;
                        d2 = fj[r].z - fi.z;
                        d0 = fmaf(-rintf(d0 * g.invLf[0]), g.Lf[0], d0);
                        d1 = fmaf(-rintf(d1 * g.invLf[1]), g.Lf[1], d1);
                        d2 = fmaf(-rintf(d2 * g.invLf[2]), g.Lf[2], d2);
                    }
                    const float r2 = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
                    const bool keep = u < u1 && u != t && r2 < lim2;
                    // survivors surely inside are stored as -(id + 1), the
                    // others as their cell-order slot for the exact test;
                    // the store is unconditional: a rejected candidate is
                    // overwritten by the next survivor, slot kLBuf - 1 takes
                    // the overflow
                    buf[min(ns, kLBuf - 1)][tl] = (SH && r2 < sure2) ? -1 - __float_as_int(fj[r].w) : u;
                    ns += keep ? 1 : 0;
                }
            }
        };
        const std::integral_constant<bool, false> no_z{};
        const std::integral_constant<bool, true> with_z{};
        auto walk = [&](auto sh_tag) {
            for (int q0 = 0; q0 < n0; ++q0) {
                int x = n0 == 3 ? cx + q0 - 1 : q0;
                float sx = 0.f;
                if (x < 0) { x += g.nc[0]; sx = -g.Lf[0]; } else if (x >= g.nc[0]) { x -= g.nc[0]; sx = g.Lf[0]; }
                for (int q1 = 0; q1 < n1; ++q1) {
                    int y = n1 == 3 ? cy + q1 - 1 : q1;
                    float sy = 0.f;
                    if (y < 0) { y += g.nc[1]; sy = -g.Lf[1]; } else if (y >= g.nc[1]) { y -= g.nc[1]; sy = g.Lf[1]; }
                    const int col = coff + (x * g.nc[1] + y) * g.nc[2];
                    if (n2 == 3) {
                        const int zlo = max(cz - 1, 0), zhi = min(cz + 1, g.nc[2] - 1);
                        scan(sh_tag, no_z, a.cell_start[col + zlo], a.cell_start[col + zhi] + a.cell_count[col + zhi],
                             sx, sy, 0.f);
                        if (cz == 0) {
                            const int cw = col + g.nc[2] - 1;
                            scan(sh_tag, with_z, a.cell_start[cw], a.cell_start[cw] + a.cell_count[cw], sx, sy,
                                 -g.Lf[2]);
                        }
                        if (cz == g.nc[2] - 1)
                            scan(sh_tag, with_z, a.cell_start[col], a.cell_start[col] + a.cell_count[col], sx, sy,
                                 g.Lf[2]);
                    } else {
                        // every cell of the column once (minimum image decides)
                        scan(sh_tag, no_z, a.cell_start[col],
                             a.cell_start[col + g.nc[2] - 1] + a.cell_count[col + g.nc[2] - 1], sx, sy, 0.f);
                    }
                }
            }
        };
        // the minimum-image form is valid on every grid; the shift form is
        // taken when it holds for every thread of the wavefront
        if (__all(shifted ? 1 : 0)) walk(std::integral_constant<bool, true>{});
        else walk(std::integral_constant<bool, false>{});
        if (ns > kLBuf - 1) {
            // too many survivors for the LDS buffer: k_search_long writes this row
            a.long_rows[atomicAdd(a.n_long, 1)] = t;
            continue;
        }

        // ---- 2: exact predicate for the survivors near the list radius,
        // accepted ids compacted in place
        const double xi = a.cell_pos[3 * (size_t)t], yi = a.cell_pos[3 * (size_t)t + 1],
                     zi = a.cell_pos[3 * (size_t)t + 2];
        int cnt = 0;
        for (int k = 0; k < ns; ++k) {
            const int u = buf[k][tl];
            if (u < 0) {
                buf[cnt++][tl] = -1 - u;
            } else if (in_range(a.cell_pos[3 * (size_t)u], a.cell_pos[3 * (size_t)u + 1],
                                a.cell_pos[3 * (size_t)u + 2], xi, yi, zi, g, a.rc2)) {
                buf[cnt++][tl] = a.cell_atoms[u];
            }
        }

        // ---- 3: sort and store
        if (cnt <= a.cap) {
            int v[kLRow];
#pragma unroll
            for (int k = 0; k < kLRow; ++k) v[k] = (k < kLBuf && k < cnt) ? buf[k < kLBuf ? k : 0][tl] : INT_MAX;
            bitonic32(v);
            // 16-byte stores (cap is a multiple of 8, so the row's last
            // partial group of four stays inside it; its padding entries lie
            // past row_count and are never read)
            int4 *out = reinterpret_cast<int4 *>(a.ell + (size_t)i * a.cap);
#pragma unroll
            for (int k = 0; k < kLRow; k += 4)
                if (k < cnt) out[k / 4] = make_int4(v[k], v[k + 1], v[k + 2], v[k + 3]);
        }
        if (BATCHED && cnt > a.cap) {
            a.row_count[i] = 0;
            atomicOr(sys_flags, 1);
        } else {
            a.row_count[i] = cnt;
        }
    }
}

// Rows listed by k_search_atoms: one wavefront per atom, the stencil's
// candidates 64 at a time through the exact predicate, compacted in order
// into LDS and rank-sorted.
constexpr int kRowCap = kMaxRow;

template <bool BATCHED>
__global__ __launch_bounds__(kWave) void k_search_long(SearchLaunch a)
{
    __shared__ int row[kRowCap];
    const int lane = threadIdx.x;
    const int nl = *a.n_long;
    for (int w = blockIdx.x; w < nl; w += gridDim.x) {
        const int t = a.long_rows[w];
        const int i = a.cell_atoms[t];
        const double xi = a.cell_pos[3 * (size_t)t], yi = a.cell_pos[3 * (size_t)t + 1],
                     zi = a.cell_pos[3 * (size_t)t + 2];
        int coff = 0;
        int *sys_flags = nullptr;
        CellGrid g;
        if constexpr (BATCHED) {
            const int sidx = a.sys_of[i];
            g = a.sys[sidx].g;
            coff = a.sys[sidx].cell_off;
            sys_flags = a.sys_status + sidx;
        } else {
            g = a.g;
        }
        const int c = a.cell_of[i] - coff;
        const int cz = c % g.nc[2], cy = (c / g.nc[2]) % g.nc[1], cx = c / (g.nc[1] * g.nc[2]);
        const int n0 = min(g.nc[0], 3), n1 = min(g.nc[1], 3), n2 = min(g.nc[2], 3);
        int cnt = 0;
        for (int q = 0; q < n0 * n1 * n2; ++q) {
            const StencilCell sc = stencil_cell(g, coff, cx, cy, cz, n0, n1, n2, q);
            const int u0 = a.cell_start[sc.cell], u1 = u0 + a.cell_count[sc.cell];
            for (int ub = u0; ub < u1; ub += kWave) {
                const int u = ub + lane;
                bool acc = false;
                if (u < u1 && u != t)
                    acc = in_range(a.cell_pos[3 * (size_t)u], a.cell_pos[3 * (size_t)u + 1],
                                   a.cell_pos[3 * (size_t)u + 2], xi, yi, zi, g, a.rc2);
                const unsigned long long m = __ballot(acc);
                const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                if (acc && cnt + below < kRowCap) row[cnt + below] = a.cell_atoms[u];
                cnt += __popcll(m);
            }
        }
        __syncthreads();
        if (cnt <= a.cap && cnt <= kRowCap) {
            int *out = a.ell + (size_t)i * a.cap;
            for (int e = lane; e < cnt; e += kWave) {
                const int v = row[e];
                int rk = 0;
                for (int q = 0; q < cnt; ++q) rk += row[q] < v;
                out[rk] = v;
            }
        }
        if (lane == 0) {
            if (BATCHED && cnt > a.cap) {
                a.row_count[i] = 0;
                atomicOr(sys_flags, 1);
            } else {
                a.row_count[i] = cnt;
            }
        }
        __syncthreads();
    }
}

// Compact list: one thread per (i, q), q < cap; the entry (i, q) of the row
// buffer (row i at i * cap) moves to jn[offsets[i] + q] when that index is
// below jn_cap (a row longer than cap was not written and is redone by the
// caller).  n_dev, when not null, holds the atom count (batches) and n is the
// capacity the grid was sized for.  total_out, when not null, receives the
// list length offsets[n].
__global__ void k_compact_list(const int *__restrict__ ell, int cap, const int *__restrict__ row_count,
                               const int *__restrict__ offsets, int n, const int *__restrict__ n_dev,
                               int *__restrict__ jn, int jn_cap, int *total_out)
{
    if (total_out && blockIdx.x == 0 && threadIdx.x == 0) *total_out = offsets[n];
    const unsigned total = (unsigned)(n_dev ? *n_dev : n) * (unsigned)cap;   // n * cap < 2^31
    const ItemRange r = xcd_items((int)((total + blockDim.x - 1) / blockDim.x));
    for (int it = r.begin; it < r.end; it += r.stride) {
        const unsigned tid = (unsigned)it * blockDim.x + threadIdx.x;
        if (tid >= total) continue;
        const int i = (int)(tid / (unsigned)cap);
        const int q = (int)(tid - (unsigned)i * (unsigned)cap);
        if (q < row_count[i]) {
            const int e = offsets[i] + q;
            if (e < jn_cap) jn[e] = ell[tid];
        }
    }
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
        if ((int)threadIdx.x < off) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + off]);
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
        if ((int)threadIdx.x < off) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + off]);
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
constexpr int kBigGridSearch = 256;   // workgroups of the long-row search

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

hipError_t launch_compact_list(const int *ell, int cap, const int *row_count, const int *offsets, int n,
                               const int *n_dev, int *jn, int jn_cap, int *total_out, hipStream_t s)
{
    const long long threads = (long long)n * cap;
    long long blocks = (threads + 255) / 256;
    if (n_dev && blocks > kBatchGrid) blocks = kBatchGrid;
    hipLaunchKernelGGL(k_compact_list, dim3((unsigned)std::max(1LL, blocks)), dim3(256), 0, s, ell, cap,
                       row_count, offsets, n, n_dev, jn, jn_cap, total_out);
    return hipGetLastError();
}

hipError_t launch_bin_atoms(const double *pos, const int *types, int n, int ntypes, const CellGrid &g,
                            int *cell_of, int *rank_in_cell, int *cell_count, int *flags, int *types_out,
                            int *near_count, hipStream_t s)
{
    // at most 1024 workgroups (each adds its near count with one atomic on a
    // single address; the grid strides over the atoms)
    const int grid = std::max(1, std::min(blocks_for(n, kBinThreads), 1024));
    hipLaunchKernelGGL(k_bin, dim3(grid), dim3(kBinThreads), 0, s, pos, types, n, ntypes, g, cell_of, rank_in_cell,
                       cell_count, flags, types_out, near_count);
    return hipGetLastError();
}

// The atoms of each cell in ascending index order: perm holds the cell
// order's slots (cell c at cell_start[c], cell_count[c] atoms, in the order
// the binning's atomics gave them); an insertion sort per cell, one thread
// per cell.  The internal numbering then depends on the positions only.
// Then, per slot t of the cell, inv[perm[t]] = t and pos_s[t] =
// pos[perm[t]] (3 doubles).
__global__ void k_sort_cells(const int *__restrict__ cell_start, const int *__restrict__ cell_count, int ncell,
                             const double *__restrict__ pos, int *__restrict__ perm, int *__restrict__ inv,
                             double *__restrict__ pos_s)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
        const int t0 = cell_start[c];
        int *seg = perm + t0;
        const int k = cell_count[c];
        for (int a = 1; a < k; ++a) {
            const int v = seg[a];
            int b = a - 1;
            while (b >= 0 && seg[b] > v) {
                seg[b + 1] = seg[b];
                --b;
            }
            seg[b + 1] = v;
        }
        for (int a = 0; a < k; ++a) {
            const int i = seg[a];
            inv[i] = t0 + a;
            pos_s[3 * (size_t)(t0 + a)] = pos[3 * (size_t)i];
            pos_s[3 * (size_t)(t0 + a) + 1] = pos[3 * (size_t)i + 1];
            pos_s[3 * (size_t)(t0 + a) + 2] = pos[3 * (size_t)i + 2];
        }
    }
}

// Row t of the renumbered list: the row of atom cell_atoms[t] with each
// neighbour named by its slot, in ascending order (rows of up to kLRow
// entries sorted in registers; a longer row places each entry by the count
// of entries below it -- slots are distinct); the type of slot t.
__global__ __launch_bounds__(256) void k_renumber_rows(const int *__restrict__ ell, const int *__restrict__ row_count,
                                                       int cap, const int *__restrict__ cell_atoms,
                                                       const int *__restrict__ inv, const int *__restrict__ types,
                                                       int n, int *__restrict__ ell_s, int *__restrict__ row_count_s,
                                                       int *__restrict__ types_s)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int i = cell_atoms[t];
        const int rc = row_count[i];
        row_count_s[t] = rc;
        types_s[t] = types[i];
        const int *row = ell + (size_t)i * cap;
        int *out = ell_s + (size_t)t * cap;
        if (rc <= kLRow) {
            // the row in 16-byte words (cap is a multiple of 8, so a word
            // starting below cap lies in the row; words past it re-read the
            // last one), then every slot lookup at once (entries past the
            // row's end look up atom 0)
            int v[kLRow];
#pragma unroll
            for (int k = 0; k < kLRow; k += 4) {
                const int4 w = *reinterpret_cast<const int4 *>(row + min(k, cap - 4));
                v[k] = w.x; v[k + 1] = w.y; v[k + 2] = w.z; v[k + 3] = w.w;
            }
#pragma unroll
            for (int k = 0; k < kLRow; ++k) v[k] = inv[k < rc ? v[k] : 0];
#pragma unroll
            for (int k = 0; k < kLRow; ++k) v[k] = k < rc ? v[k] : INT_MAX;
            bitonic32(v);
            // 16-byte stores, words starting below cap only (entries past
            // row_count are padding, never read)
#pragma unroll
            for (int k = 0; k < kLRow; k += 4)
                if (k < rc && k < cap) *reinterpret_cast<int4 *>(out + k) = make_int4(v[k], v[k + 1], v[k + 2], v[k + 3]);
        } else {
            for (int e = 0; e < rc; ++e) {
                const int u = inv[row[e]];
                int below = 0;
                for (int f = 0; f < rc; ++f) below += inv[row[f]] < u ? 1 : 0;
                out[below] = u;
            }
        }
    }
}

hipError_t launch_renumber_rows(const int *ell, const int *row_count, int cap, const int *cell_atoms,
                                const int *cell_start, const int *cell_count, int ncell, const int *types,
                                const double *pos, int n, int *perm, int *inv, int *ell_s, int *row_count_s,
                                int *types_s, double *pos_s, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(perm, cell_atoms, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    const int cgrid = std::max(1, std::min(blocks_for(ncell, 256), 4096));
    hipLaunchKernelGGL(k_sort_cells, dim3(cgrid), dim3(256), 0, s, cell_start, cell_count, ncell, pos, perm, inv,
                       pos_s);
    const int grid = std::max(1, std::min(blocks_for(n, 256), 4096));
    hipLaunchKernelGGL(k_renumber_rows, dim3(grid), dim3(256), 0, s, ell, row_count, cap, perm, inv, types, n,
                       ell_s, row_count_s, types_s);
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

hipError_t launch_scatter_cells(const ScatterLaunch &a, int grid_cap, hipStream_t s)
{
    int grid = blocks_for(a.n, 256);
    if (a.dims) {
        grid = std::min(grid, grid_cap);
        hipLaunchKernelGGL(k_scatter<true>, dim3(std::max(1, grid)), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_scatter<false>, dim3(std::max(1, grid)), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_search(const SearchLaunch &a, int grid_cap, hipStream_t s)
{
    if (a.cap < 8 || a.cap % 8 != 0) return hipErrorInvalidValue;   // rows are written 16 bytes at a time
    int grid = std::max(1, blocks_for(a.n, kSearchThreads));
    if (a.dims) {
        grid = std::min(grid, grid_cap);
        hipLaunchKernelGGL(k_search_atoms<true>, dim3(grid), dim3(kSearchThreads), 0, s, a);
        hipLaunchKernelGGL(k_search_long<true>, dim3(kBigGridSearch), dim3(kWave), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_search_atoms<false>, dim3(grid), dim3(kSearchThreads), 0, s, a);
        hipLaunchKernelGGL(k_search_long<false>, dim3(kBigGridSearch), dim3(kWave), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace tsf
