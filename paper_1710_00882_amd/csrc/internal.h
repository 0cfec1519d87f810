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
    real c2d2;        // c^2 / d^2
    real d2;          // d^2
    real two_c2;      // 2 c^2
    real h, gamma;
    real R, Rin;      // R, R - D
    real half_pi_D;   // pi / (2 D)
    real m;           // 1 or 3
    // Error-compensated pair constants: ln A = lnA + lnA_lo, lambda1 =
    // lam1 + lam1_lo (likewise B, lambda2), each lo part the rounding error
    // of its hi part in this precision (zero in FP64).
    real lnA, lnA_lo, lam1_lo;
    real lnB, lnB_lo, lam2_lo;
    real R_lo, half_pi_D_lo;  // likewise for the switching-function argument
    real pad;
};

// FP64 quantities used by both precisions (membership tests and the
// zeta -> b power in log form).
struct ParamX {
    double cutsq;     // (R + D)^2
    double logbeta;   // log(beta) (unused when beta == 0)
    double eta;
    double inv2eta;   // 1 / (2 eta)
};

struct DeviceTable {
    int ntypes;
    const ParamR<float> *pf;    // ntypes^3 entries
    const ParamR<double> *pd;   // ntypes^3 entries
    const ParamX *px;           // ntypes^3 entries
    const double *packsq;       // ntypes^2, symmetric: packing radius^2 of a (ti, tn) entry
};

// Flags raised by kernels (bitwise OR into a device int).
enum : int { kFlagOverflow = 1, kFlagStale = 2 };

constexpr int kRecCap = 32;   // packed-neighbour records per atom (more: E_OVERFLOW)
constexpr int kBigGrid = 64;  // workgroups of the dropped-atom fixup kernel

struct PackLaunch {
    const double *pos;          // n x 3
    const int *types;           // n
    const int *offsets;         // n + 1 (CSR, int32, internal row order)
    const int2 *jr;             // S: (neighbour j, entry of i in row j)
    int n;
    double L[3], invL[3];
    void *recs;                 // n x kRecCap packed records
    int *pcount;                // n: records per atom
    int *slotpos;               // S: rank among the row's kept entries, -1 not kept, -2 beyond cap
    double *own;                // n x 3 (zeroed for dropped atoms only)
    int *flags;
    int *drop_list;             // n: atoms with more kept neighbours than kRecCap
    int *drop_count;            // reset to 0 here
    const double *pos_build;    // n x 3 positions of the last build (stale check)
    double stale_sq;            // (skin / 2)^2
};

struct ComputeLaunch {
    const int *types;           // n
    const void *recs;           // n x kRecCap packed records
    const int *pcount;          // n
    const int *slotpos;         // S
    int n;
    double *own;                // n x 3: force from the terms of each centre atom
    double *planes;             // kRecCap x n x 3: plane k of atom j = force from its k-th kept neighbour's terms
    double *partials;           // grid x 8
    long long *counters;        // grid x 2 (pairs, triplets)
    int atoms_per_batch;        // nominal atoms per batch (<= kWave)
};

// Launchers (compute.hip).  grids = {pack, compute} workgroup counts plus
// kBigGrid for the fixup kernel.
void compute_grids(bool mixed, bool one_type, int n, int atoms_per_batch, int grids[3]);
size_t record_bytes(bool mixed);
hipError_t launch_pack(const PackLaunch &a, const DeviceTable &t, bool mixed, int grid, hipStream_t s);
hipError_t launch_compute(const ComputeLaunch &a, const DeviceTable &t, bool mixed,
                          int grid, hipStream_t s);
hipError_t launch_fixup_dropped(const int *offsets, const int2 *jr, const int *slotpos,
                                const int *drop_list, const int *drop_count, int n, double *planes,
                                hipStream_t s);
hipError_t launch_finalize(const double *partials, const long long *counters, int grid,
                           double *out7, long long *counts_out, hipStream_t s);
hipError_t launch_fill_zero(double *p, size_t count, hipStream_t s);
hipError_t launch_gather_forces(const int *pcount, const double *planes, const double *own, int n,
                                double *forces, hipStream_t s);

// Neighbour build (neighbors.hip)
struct CellGrid {
    int nc[3];
    double L[3];
    double cell_w[3];
};
hipError_t launch_bin_atoms(const double *pos, int n, const CellGrid &g, int *cell_of,
                            int *rank_in_cell, int *cell_count, hipStream_t s);
hipError_t launch_scatter_cells(const double *pos, int n, const int *cell_of,
                                const int *rank_in_cell, const int *cell_start,
                                int *cell_atoms, double *cell_pos, hipStream_t s);
hipError_t launch_search(const double *pos, int n, const CellGrid &g, double rcut,
                         const int *cell_of, const int *cell_start, const int *cell_count,
                         const int *cell_atoms, const double *cell_pos, int cap, int *ell,
                         float *ell_r2, int *row_count, hipStream_t s);
hipError_t launch_sort_rows(const int *ell, const float *ell_r2, int cap, const int *row_count,
                            const int *offsets, int n, int *idx, int2 *jr, int *perm, hipStream_t s);
// jr[e].y for internal entry e = (i, j): the internal entry of (j, i) (the
// list is symmetric).  Sets *flags |= 4 if some reverse entry is missing.
hipError_t launch_reverse_map(const int *offsets, const int *idx, const int *perm, int n, int2 *jr,
                              int *flags, hipStream_t s);
hipError_t launch_check_inputs(const double *pos, const int *types, int n, int ntypes,
                               int *flags, hipStream_t s);

// Exclusive scan of n int32 values; out[n] receives the total.  tmp must hold
// scan_tmp_size(n) ints.  Also writes the maximum input to *max_out when
// max_out is not null.
size_t scan_tmp_size(int n);
hipError_t launch_exclusive_scan(const int *in, int *out, int n, int *tmp, int *max_out,
                                 hipStream_t s);

}  // namespace tsf
