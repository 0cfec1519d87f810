// Cell-list neighbour build (Section 2: full per-atom list including the
// skin atoms).  Every kernel here evaluates the inclusion predicate with the
// same rounding sequence as its definition:
//   per axis  t = x_j - x_i;  s = rint(t / L);  d = fma(-s, L, t)
//   r^2 = fma(dz, dz, fma(dy, dy, dx * dx));  include j iff r^2 < rcut^2
// with FP contraction disabled, so the lists are bit-identical to any other
// implementation of that predicate.
//
// Steps: input check -> bin atoms to cells (count + rank per cell) ->
// exclusive scan of cell counts -> scatter atom ids and positions into cell
// order -> one thread per atom scans the unique neighbouring cells into a
// fixed-capacity row buffer -> scan of row counts (CSR offsets) -> each row is
// rank-sorted by 16 lanes into its CSR slot (public order by j, internal
// order nearest-first) -> reverse-entry map of the internal order.
#include "internal.h"

#pragma clang fp contract(off)

namespace tsf {

namespace {

__device__ inline int cell_index(double x, double L, double w, int nc)
{
    double u = x - L * floor(x / L);
    int c = (int)floor(u / w);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_check_inputs(const double *__restrict__ pos, const int *__restrict__ types,
                               int n, int ntypes, int *flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int f = 0;
    for (int a = 0; a < 3; ++a)
        if (!isfinite(pos[3 * (size_t)i + a])) f |= 1;
    int t = types[i];
    if (t < 0 || t >= ntypes) f |= 2;
    if (f) atomicOr(flags, f);
}

__global__ void k_bin(const double *__restrict__ pos, int n, CellGrid g, int *__restrict__ cell_of,
                      int *__restrict__ rank, int *__restrict__ count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *p = pos + 3 * (size_t)i;
    int cx = cell_index(p[0], g.L[0], g.cell_w[0], g.nc[0]);
    int cy = cell_index(p[1], g.L[1], g.cell_w[1], g.nc[1]);
    int cz = cell_index(p[2], g.L[2], g.cell_w[2], g.nc[2]);
    int c = (cx * g.nc[1] + cy) * g.nc[2] + cz;
    cell_of[i] = c;
    rank[i] = atomicAdd(&count[c], 1);
}

__global__ void k_scatter(const double *__restrict__ pos, int n, const int *__restrict__ cell_of,
                          const int *__restrict__ rank, const int *__restrict__ cell_start,
                          int *__restrict__ cell_atoms, double *__restrict__ cell_pos)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int slot = cell_start[cell_of[i]] + rank[i];
    cell_atoms[slot] = i;
    cell_pos[3 * (size_t)slot + 0] = pos[3 * (size_t)i + 0];
    cell_pos[3 * (size_t)slot + 1] = pos[3 * (size_t)i + 1];
    cell_pos[3 * (size_t)slot + 2] = pos[3 * (size_t)i + 2];
}

__device__ inline double image_component(double xj, double xi, double L)
{
    double t = xj - xi;
    double s = rint(t / L);
    return fma(-s, L, t);
}

__global__ void k_search(const double *__restrict__ pos, int n, CellGrid g, double rc2,
                         const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                         const int *__restrict__ cell_count, const int *__restrict__ cell_atoms,
                         const double *__restrict__ cpos, int cap, int *__restrict__ ell,
                         float *__restrict__ ell_r2, int *__restrict__ row_count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = pos[3 * (size_t)i], yi = pos[3 * (size_t)i + 1], zi = pos[3 * (size_t)i + 2];
    int c = cell_of[i];
    int c2 = c % g.nc[2];
    int c1 = (c / g.nc[2]) % g.nc[1];
    int c0 = c / (g.nc[2] * g.nc[1]);
    // unique neighbouring cells per axis: {-1,0,1} when nc >= 3, {0,1} when 2, {0} when 1
    int lo0 = g.nc[0] >= 3 ? -1 : 0, hi0 = g.nc[0] >= 3 ? 1 : g.nc[0] - 1;
    int lo1 = g.nc[1] >= 3 ? -1 : 0, hi1 = g.nc[1] >= 3 ? 1 : g.nc[1] - 1;
    int lo2 = g.nc[2] >= 3 ? -1 : 0, hi2 = g.nc[2] >= 3 ? 1 : g.nc[2] - 1;
    int cnt = 0;
    int *row = ell + (size_t)i * cap;
    float *row_r2 = ell_r2 + (size_t)i * cap;
    for (int o0 = lo0; o0 <= hi0; ++o0) {
        int x = c0 + o0; x += (x < 0) ? g.nc[0] : 0; x -= (x >= g.nc[0]) ? g.nc[0] : 0;
        for (int o1 = lo1; o1 <= hi1; ++o1) {
            int y = c1 + o1; y += (y < 0) ? g.nc[1] : 0; y -= (y >= g.nc[1]) ? g.nc[1] : 0;
            for (int o2 = lo2; o2 <= hi2; ++o2) {
                int z = c2 + o2; z += (z < 0) ? g.nc[2] : 0; z -= (z >= g.nc[2]) ? g.nc[2] : 0;
                int cc = (x * g.nc[1] + y) * g.nc[2] + z;
                int s0 = cell_start[cc], s1 = s0 + cell_count[cc];
                for (int s = s0; s < s1; ++s) {
                    int j = cell_atoms[s];
                    if (j == i) continue;
                    double dx = image_component(cpos[3 * (size_t)s + 0], xi, g.L[0]);
                    double dy = image_component(cpos[3 * (size_t)s + 1], yi, g.L[1]);
                    double dz = image_component(cpos[3 * (size_t)s + 2], zi, g.L[2]);
                    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                    if (r2 < rc2) {
                        if (cnt < cap) {
                            row[cnt] = j;
                            row_r2[cnt] = (float)r2;
                        }
                        ++cnt;
                    }
                }
            }
        }
    }
    row_count[i] = cnt;
}

// 16 lanes per row: each lane takes elements lane, lane+16, ... and places
// each by its rank within the row (row entries are distinct atom ids), twice:
// by j for the public list, and nearest-first (r^2 at build, ties by j) for
// the internal order the compute kernels walk; perm maps a public position
// to the internal position of the same entry.
__global__ void k_sort_rows(const int *__restrict__ ell, const float *__restrict__ ell_r2, int cap,
                            const int *__restrict__ row_count, const int *__restrict__ offsets, int n,
                            int *__restrict__ idx, int2 *__restrict__ jr, int *__restrict__ perm)
{
    int r = blockIdx.x * (blockDim.x / 16) + threadIdx.x / 16;
    int l = threadIdx.x % 16;
    if (r >= n) return;
    int cnt = row_count[r];
    if (cnt > cap) return;   // never launched in this state (the build retries first)
    const int *row = ell + (size_t)r * cap;
    const float *row_r2 = ell_r2 + (size_t)r * cap;
    int base = offsets[r];
    for (int e = l; e < cnt; e += 16) {
        const int v = row[e];
        const float d = row_r2[e];
        int rank_j = 0, rank_d = 0;
        for (int m = 0; m < cnt; ++m) {
            const int w = row[m];
            const float dm = row_r2[m];
            rank_j += w < v;
            rank_d += (dm < d) || (dm == d && w < v);
        }
        idx[base + rank_j] = v;
        jr[base + rank_d] = make_int2(v, -1);
        perm[base + rank_j] = base + rank_d;
    }
}

// jr[e].y for internal entry e = (i, j): the internal position of entry
// (j, i), found by binary search of i in j's public (sorted) row and mapped
// through perm.  The inclusion predicate is symmetric (negating t negates s
// and d exactly), so the entry exists; a missing one raises flag 4.
__global__ void k_reverse_map(const int *__restrict__ offsets, const int *__restrict__ idx,
                              const int *__restrict__ perm, int n, int2 *__restrict__ jr, int *flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int e = offsets[i]; e < offsets[i + 1]; ++e) {
        const int j = jr[e].x;
        int lo = offsets[j], hi = offsets[j + 1] - 1, at = -1;
        while (lo <= hi) {
            int mid = (lo + hi) >> 1;
            int v = idx[mid];
            if (v == i) { at = mid; break; }
            if (v < i) lo = mid + 1; else hi = mid - 1;
        }
        if (at < 0) {
            atomicOr(flags, 4);
            jr[e].y = e;
        } else {
            jr[e].y = perm[at];
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

hipError_t launch_reverse_map(const int *offsets, const int *idx, const int *perm, int n, int2 *jr,
                              int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_reverse_map, dim3(blocks_for(n, 256)), dim3(256), 0, s, offsets, idx, perm, n,
                       jr, flags);
    return hipGetLastError();
}

hipError_t launch_check_inputs(const double *pos, const int *types, int n, int ntypes,
                               int *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_inputs, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos, types, n,
                       ntypes, flags);
    return hipGetLastError();
}

hipError_t launch_bin_atoms(const double *pos, int n, const CellGrid &g, int *cell_of,
                            int *rank_in_cell, int *cell_count, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos, n, g, cell_of,
                       rank_in_cell, cell_count);
    return hipGetLastError();
}

hipError_t launch_scatter_cells(const double *pos, int n, const int *cell_of,
                                const int *rank_in_cell, const int *cell_start,
                                int *cell_atoms, double *cell_pos, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, pos, n, cell_of,
                       rank_in_cell, cell_start, cell_atoms, cell_pos);
    return hipGetLastError();
}

hipError_t launch_search(const double *pos, int n, const CellGrid &g, double rcut,
                         const int *cell_of, const int *cell_start, const int *cell_count,
                         const int *cell_atoms, const double *cell_pos, int cap, int *ell,
                         float *ell_r2, int *row_count, hipStream_t s)
{
    hipLaunchKernelGGL(k_search, dim3(blocks_for(n, 128)), dim3(128), 0, s, pos, n, g,
                       rcut * rcut, cell_of, cell_start, cell_count, cell_atoms, cell_pos, cap,
                       ell, ell_r2, row_count);
    return hipGetLastError();
}

hipError_t launch_sort_rows(const int *ell, const float *ell_r2, int cap, const int *row_count,
                            const int *offsets, int n, int *idx, int2 *jr, int *perm, hipStream_t s)
{
    hipLaunchKernelGGL(k_sort_rows, dim3(blocks_for(n, 16)), dim3(256), 0, s, ell, ell_r2, cap,
                       row_count, offsets, n, idx, jr, perm);
    return hipGetLastError();
}

}  // namespace tsf
