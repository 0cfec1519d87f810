// Internal declarations shared by the translation units of libtersoff.so.
// Nothing here is part of the public C ABI (include/tersoff.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tsf {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxTypes = 4;

// Per-entry parameters in the working precision of a kernel, with the
// derived constants the kernels use (no divisions left on the hot path).
template <typename real>
struct ParamR {
    real A, B, lam1, lam2;
    real lam3;        // lambda3
    real lam3m;       // lambda3^m (m = 1 or 3)
    real c2d2;        // gamma c^2 / d^2
    real d2;          // d^2
    real two_c2;      // 2 gamma c^2
    real h, gamma;
    real Rc, Rin;     // R + D (the cutoff), R - D
    real qpi_D;       // pi / (4 D)
    real m;           // 1 or 3
    // Error-compensated pair constants: ln A = lnA + lnA_lo, lambda1 =
    // lam1 + lam1_lo (likewise B, lambda2), each lo part the rounding error
    // of its hi part in this precision (zero in FP64).
    real lnA, lnA_lo, lam1_lo;
    real lnB, lnB_lo, lam2_lo;
    real Rc_lo, qpi_D_lo;     // likewise for the switching-function argument
    real beta;                // beta (the all-FP32 path forms ln(beta zeta) from the product)
};

// FP64 quantities used by both precisions (membership tests and the
// zeta -> b power in log form).
struct ParamX {
    double cutsq;     // (R + D)^2
    double logbeta;   // log(beta) (-inf when beta == 0)
    double eta;
    double inv2eta;   // 1 / (2 eta)
    double A, B, lam1, lam2;   // the mixed path scales its pair exponentials and sums the pair force in FP64
};

struct DeviceTable {
    int ntypes;
    const ParamR<float> *pf;    // ntypes^3 entries
    const ParamR<double> *pd;   // ntypes^3 entries
    const ParamX *px;           // ntypes^3 entries
    const double *packsq;       // ntypes^2, symmetric: packing radius^2 of a (ti, tn) entry
    int lam3_zero;              // one species with lambda3 = 0 (the exponential factor is 1)
    int sym3;                   // three-body parameters of (ti, tj, tk) equal those of (ti, tk, tj)
};

// Cell grid of one periodic box (cells at least the list radius wide).
struct CellGrid {
    int nc[3];
    double L[3];
    double invL[3];
    double cell_w[3];
    float Lf[3], invLf[3];   // single-precision copies for the conservative pre-test
    float Lsum;              // Lf[0] + Lf[1] + Lf[2]
};
// One configuration of a batch: its box and cell grid, and where its atoms
// and cells start in the batch's concatenated arrays.
struct SysDesc {
    CellGrid g;
    int atom_off, natoms;
    int cell_off, pad;
};

// Sizes of the batch in flight, read by the kernels from device memory so
// that one captured launch sequence serves batches of any size up to the
// capacities its grids were sized for.
struct BatchDims {
    int n_atoms, n_cells, n_sys, pad;
};

constexpr int kBatchGrid = 2048;   // workgroups of the grid-stride kernels of a batch

// Workgroups are dealt to the 8 XCDs of the chip round-robin (workgroup b on
// XCD b mod 8), each XCD with its own L2.  Give every XCD a contiguous range
// of work items so that neighbouring atoms -- which share position, record
// and force cache lines -- are handled under the same L2.  Any other
// placement only costs locality, never correctness.
struct ItemRange {
    int begin, end, stride;
};

__device__ __forceinline__ ItemRange xcd_items(int nitems)
{
    const int G = gridDim.x;
    if (G < 8) return {(int)blockIdx.x, nitems, G};
    const int x = blockIdx.x & 7, l = blockIdx.x >> 3;
    const int gx = (G - x + 7) / 8;          // workgroups on this XCD
    const int per = (nitems + 7) / 8;
    const int b0 = x * per;
    return {b0 + l, min(nitems, b0 + per), gx};
}

// Flags raised by kernels (bitwise OR into a device int).  kFlagAsym: a
// centre kept a neighbour whose kept list (shorter than kRecCap) lacks it.
enum : int { kFlagOverflow = 1, kFlagStale = 2, kFlagAsym = 4 };

constexpr int kRecCap = 32;   // packed-neighbour records per atom (more: E_OVERFLOW)
// Kept-neighbour lists of N atoms in one buffer of (kKeptFast + kRecCap) N
// ints: the first kKeptFast entries of atom m at kept[m * kKeptFast] (one
// 32-byte block, -1 after the last entry), entries kKeptFast .. kRecCap - 1
// at kept_more[m * kRecCap + q], kept_more = kept + kKeptFast N (-1 after the
// last when the list is shorter than kRecCap).
constexpr int kKeptFast = 8;
constexpr int kFusedRowCap = 64;   // longest neighbour row of the fused packing (one 64-bit kept mask)
constexpr int kBigGrid = 64;  // workgroups of the dropped-atom fixup kernel

struct PackLaunch {
    const double *pos;          // n x 3
    const int *types;           // n
    const int *row_count;       // n: list length of each atom
    const int *ell;             // neighbour rows (sorted), row i at i * cap, row_count[i] entries
    int cap;                    // row stride
    int n;
    double L[3], invL[3];
    void *recs;                 // packed records: region of B * kRecCap per batch of B atoms
    float *rlo;                 // float records: per record, r - (the compute kernel's FP32 r), or null
    int *pcount;                // n: records per atom
    int *kept;                  // n x kKeptFast: kept-neighbour lists (first entries)
    int *kept_more;             // n x kRecCap: kept-neighbour lists (entries kKeptFast ..)
    double *own;                // n x 3 (zeroed for dropped atoms only)
    int *flags;
    int *drop_list;             // n: atoms with more kept neighbours than kRecCap
    int *drop_count;            // 0 on entry (the gather / batch set-up kernels reset it)
    const double *pos_build;    // n x 3 positions of the last build (stale check)
    double stale_sq;            // (skin / 2)^2
    int atoms_per_batch;        // B: centre atoms per batch (<= kWave), shared with the compute kernel
    // batches of systems (null for one system): atom count, box of each atom's system
    const int *n_dev;
    const SysDesc *sys;
    const int *sys_of;
};

struct ComputeLaunch {
    const int *types;           // n
    const void *recs;           // packed records (batch regions)
    const float *rlo;           // float records: FP64 r minus FP32 r, per record (same index)
    const int *pcount;          // n
    const int *kept;            // kept-neighbour lists of plane_stride atoms (kept_more follows)
    int n;
    double *own;                // n x 3: force from the terms of each centre atom
    void *planes;               // kRecCap x n x 3: plane k of atom j = force from its k-th kept neighbour's
                                // terms (float for the mixed and single paths, double for FP64)
    double *partials;           // grid x 8 (E, virial, kFlagAsym as a double)
    long long *counters;        // grid x 2 (pairs, triplets)
    int atoms_per_batch;        // nominal atoms per batch (<= kWave)
    int plane_stride;           // atoms per force plane (n, or the batch capacity)
    // batches of systems (null for one system): atom count; per-atom energy
    // and virial (8 doubles per atom) in place of the per-workgroup partials
    const int *n_dev;
    double *eatom;
    // one system, atomic scatter (the comparison point of the force planes):
    // when not null, every force term is added with FP64 atomics into this
    // n x 3 array (zeroed beforehand), and own / planes / kept are not used
    double *forces_atomic;
    // one system, fused packing (rows not null): the kernel packs each group's
    // rows itself (no records, kept lists or counts in memory); the force on
    // atom m from centre i goes to plane e of m, e = position of i in m's row
    // (< kFusedRowCap), and kmask[m] marks the row positions whose centres
    // keep m (the planes k_gather_rows adds)
    const int *rows;            // neighbour rows (stride cap, sorted)
    const unsigned char *rev;   // same layout: position of the centre in that neighbour's row
    const int *row_count;       // n
    int cap;
    const double *pos;          // n x 3
    const double *pos_build;    // n x 3: positions of the last build (stale check)
    double L[3], invL[3];
    double stale_sq;
    int *flags;
    unsigned long long *kmask;  // n
};

// Launchers (compute.hip).  grids = {pack, compute} workgroup counts,
// kBigGrid for the fixup kernel, and the compute grid of the fused packing
// (one system; 0 for batches).
// Precisions (the values of tersoff_precision).
enum : int { kPrecFP64 = 0, kPrecMixed = 1, kPrecSingle = 2, kNumPrec = 3 };

void compute_grids(int prec, const DeviceTable &t, bool batched, int n, int atoms_per_batch, int grids[4]);
size_t record_bytes(int prec);
// Bytes of a record region of `slots` records, the per-record r corrections
// of the float records included (placed after the records; rlo_of gives them).
size_t record_region_bytes(int prec, size_t slots);
float *rlo_of(void *recs, int prec, size_t slots);
hipError_t launch_pack(const PackLaunch &a, const DeviceTable &t, int prec, int grid, hipStream_t s);
hipError_t launch_compute(const ComputeLaunch &a, const DeviceTable &t, int prec,
                          int grid, hipStream_t s);
// The lane-per-triplet kernel (one system, FP64 or mixed, force planes) on at
// most max_grid workgroups; *grid_used: the workgroups launched (partial sums).
hipError_t launch_compute_triplet(const ComputeLaunch &a, const DeviceTable &t, int prec, int max_grid,
                                  hipStream_t s, int *grid_used);
// Force planes hold float for the mixed and single paths, double for FP64.
hipError_t launch_fixup_dropped(const int *ell, int cap, const int *row_count, const int *kept,
                                const int *kept_more, const int *drop_list, const int *drop_count,
                                int plane_stride, int prec, void *planes, hipStream_t s);
hipError_t launch_fill_zero(double *p, size_t count, hipStream_t s);
// The sum of the compute kernel's per-workgroup partials (grid rows of 8
// doubles and 2 counts) into out7 / counts_out; kFlagAsym into *flags when a
// partial carries it.  partials == nullptr: none (batched path).
struct FinalizeArgs {
    const double *partials;
    const long long *counters;
    int grid;
    double *out;
    long long *counts;
    int *flags;
};
constexpr int kGatherThreads = 256;
// drop_count, when not null, is reset to 0 (the dropped-atom list is empty
// for the next evaluation); fin.partials, when not null, adds the sum of the
// partials (one extra workgroup).
// perm, when not null: forces of atom m stored at the caller's index perm[m].
hipError_t launch_gather_forces(const int *pcount, int prec, const void *planes, const double *own, int n,
                                const int *n_dev, int plane_stride, double *forces, const int *perm,
                                int *drop_count, const FinalizeArgs &fin, hipStream_t s);
// Per-system sums of the per-atom energy / virial of a batch and status bits
// (1: a neighbour row over capacity, 2: an atom over the record capacity):
// out[8 s + c] = E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz, status.
hipError_t launch_reduce_systems(const SysDesc *sys, const BatchDims *dims, int max_sys, const double *eatom,
                                 const int *drop_list, const int *drop_count, const int *sys_status,
                                 double *out, hipStream_t s);
hipError_t launch_fill_zero_int(int *p, size_t count, hipStream_t s);
// Fused packing: the force on each atom m from the planes its row's kept
// centres wrote (kmask[m], in row order) plus its own; fin as above.
hipError_t launch_gather_rows(const unsigned long long *kmask, int prec, const void *planes, const double *own,
                              int n, int plane_stride, double *forces, const int *perm, const FinalizeArgs &fin,
                              hipStream_t s);
// posp[t] = pos[perm[t]]; out[perm[t]] = in[t] (n atoms, 3 doubles each).
hipError_t launch_permute_pos(const double *pos, const int *perm, int n, double *posp, hipStream_t s);
hipError_t launch_unpermute3(const double *in, const int *perm, int n, double *out, hipStream_t s);
// rev[i cap + e] = position of i in the row of its neighbour ell[i cap + e],
// for the rows of n atoms (row_count, at most cap <= 256 entries each,
// sorted); kFlagAsym into *flags when a neighbour's row lacks i.
hipError_t launch_reverse_index(const int *ell, const int *row_count, int cap, int n, unsigned char *rev,
                                int *flags, hipStream_t s);

// Neighbour build (neighbors.hip)
// Cells and in-cell ranks of the atoms; types copied to types_out; into
// *near_count, the consecutive atoms (i, i + 1), i mod 64 != 63, in the same
// or adjacent cells (how coherent in space the caller's atom order is).
hipError_t launch_bin_atoms(const double *pos, const int *types, int n, int ntypes, const CellGrid &g,
                            int *cell_of, int *rank_in_cell, int *cell_count, int *flags, int *types_out,
                            int *near_count, hipStream_t s);
// The internal numbering: perm[t] = the atom of slot t, the cell order
// (cell_atoms, cells at cell_start with cell_count atoms) with each cell's
// atoms in ascending index order; inv (n ints) receives each atom's slot;
// row t of ell_s / row_count_s is the row of atom perm[t] with its
// neighbours' slots in ascending order, types_s[t] its type, pos_s[t] its
// position in pos (3 doubles).  Rows at stride cap.
hipError_t launch_renumber_rows(const int *ell, const int *row_count, int cap, const int *cell_atoms,
                                const int *cell_start, const int *cell_count, int ncell, const int *types,
                                const double *pos, int n, int *perm, int *inv, int *ell_s, int *row_count_s,
                                int *types_s, double *pos_s, hipStream_t s);
// Cell-order copies of the atoms (ids, FP64 positions, wrapped FP32
// positions with the id in the fourth word).  Batches: dims and the
// per-atom system set, n the capacity the grid is sized for.
struct ScatterLaunch {
    const double *pos;
    int n;
    const int *cell_of, *rank, *cell_start;
    int *cell_atoms;
    double *cell_pos;
    float4 *cell_posf;
    double *pos_copy;                // when not null: a copy of pos (atom order)
    int *slot_cell;                  // cell of each cell-order slot
    CellGrid g;                      // one system
    const SysDesc *sys;              // batches
    const int *sys_of;
    const BatchDims *dims;
};
hipError_t launch_scatter_cells(const ScatterLaunch &a, int grid_cap, hipStream_t s);

// Neighbour rows (sorted, stride cap, cap a multiple of 8; a row's last
// group of four entries may carry padding past row_count) of every atom;
// rows longer than cap are not written (row_count holds the true length, or 0 with bit 1 of the
// system's status in a batch).  long_rows / n_long: scratch for rows too long
// for the first pass (n_long must be 0 on entry).
// Entries past the end of the cell-order FP32 positions that the search may
// load (and discard); allocations of cell_posf hold n + kPosPad entries.
constexpr int kPosPad = 4;
struct SearchLaunch {
    CellGrid g;
    const SysDesc *sys;
    const int *sys_of;
    const BatchDims *dims;
    int n;
    double rc2;
    float rcs;
    const int *cell_start, *cell_count, *cell_atoms, *cell_of;
    const int *slot_cell;            // cell of each cell-order slot
    const double *cell_pos;
    const float4 *cell_posf;
    int cap;
    int *ell, *row_count;
    int *long_rows, *n_long;
    int *sys_status;
};
hipError_t launch_search(const SearchLaunch &a, int grid_cap, hipStream_t s);
// Compact list from the row buffer (row i at i * cap): jn[offsets[i] + q] =
// ell[i * cap + q] for q < row_count[i], entries at or past jn_cap skipped;
// *total_out = offsets[n] when total_out is not null.
hipError_t launch_compact_list(const int *ell, int cap, const int *row_count, const int *offsets, int n,
                               const int *n_dev, int *jn, int jn_cap, int *total_out, hipStream_t s);
// Batched build: binning of every system's atoms into its own cells.
hipError_t launch_bin_systems(const double *pos, const int *sys_of, const SysDesc *sys, const BatchDims *dims,
                              int max_atoms, int *cell_of, int *rank_in_cell, int *cell_count, hipStream_t s);
constexpr int kMaxRow = 256;    // longest neighbour row the build supports

// Exclusive scan of n int32 values; out[n] receives the total.  tmp must hold
// scan_tmp_size(n) ints.  Also writes the maximum input to *max_out when
// max_out is not null.
size_t scan_tmp_size(int n);
hipError_t launch_exclusive_scan(const int *in, int *out, int n, int *tmp, int *max_out,
                                 hipStream_t s);

// Molecular-dynamics driver kernels (md.hip).
hipError_t launch_md_kick(double *vel, const double *f, const int *types, const double *inv_mass, double c, int n,
                          hipStream_t s);
hipError_t launch_md_drift(double *pos, const double *vel, double dt, int n, hipStream_t s);
hipError_t launch_md_displaced(const double *pos, const double *pos_build, double lim2, int n, int *flag,
                               hipStream_t s);
int md_kinetic_blocks();
hipError_t launch_md_kinetic(const double *vel, const int *types, const double *mass, int n, double *partials,
                             hipStream_t s);

}  // namespace tsf
