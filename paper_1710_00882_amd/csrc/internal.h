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
    const int *row_count;       // n: list length of each atom
    const int *jn;              // n x cap: sorted neighbour rows (row i at i * cap)
    const int *rv;              // n x cap: entry of (j, i) for entry (i, j)
    int cap;
    int n;
    double L[3], invL[3];
    void *recs;                 // packed records: region of B * kRecCap per batch of B atoms
    int *pcount;                // n: records per atom
    signed char *slotpos;       // n x cap: rank among the row's kept entries, -1 not kept, -2 beyond kRecCap
    double *own;                // n x 3 (zeroed for dropped atoms only)
    int *flags;
    int *drop_list;             // n: atoms with more kept neighbours than kRecCap
    int *drop_count;            // reset to 0 here
    const double *pos_build;    // n x 3 positions of the last build (stale check)
    double stale_sq;            // (skin / 2)^2
    int atoms_per_batch;        // B: centre atoms per batch (<= kWave), shared with the compute kernel
};

struct ComputeLaunch {
    const int *types;           // n
    const void *recs;           // packed records (batch regions)
    const int *pcount;          // n
    const signed char *slotpos; // n x cap
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
hipError_t launch_fixup_dropped(const int *row_count, const int *jn, const int *rv, int cap,
                                const signed char *slotpos, const int *drop_list, const int *drop_count,
                                int n, double *planes, hipStream_t s);
hipError_t launch_finalize(const double *partials, const long long *counters, int grid,
                           double *out7, long long *counts_out, hipStream_t s);
hipError_t launch_fill_zero(double *p, size_t count, hipStream_t s);
hipError_t launch_gather_forces(const int *pcount, const double *planes, const double *own, int n,
                                double *forces, hipStream_t s);

// Neighbour build (neighbors.hip)
struct CellGrid {
    int nc[3];
    double L[3];
    double invL[3];
    double cell_w[3];
    float Lf[3], invLf[3];   // single-precision copies for the conservative pre-test
    float Lsum;              // Lf[0] + Lf[1] + Lf[2]
};
hipError_t launch_bin_atoms(const double *pos, const int *types, int n, int ntypes, const CellGrid &g,
                            int *cell_of, int *rank_in_cell, int *cell_count, int *flags, hipStream_t s);
hipError_t launch_scatter_cells(const double *pos, int n, const int *cell_of,
                                const int *rank_in_cell, const int *cell_start,
                                int *cell_atoms, double *cell_pos, hipStream_t s);
hipError_t launch_search(const CellGrid &g, double rcut, const int *cell_start, const int *cell_count,
                         const int *cell_atoms, const double *cell_pos, int ncell, int cap, int *ell,
                         int *row_count, hipStream_t s);
// rv[e] for entry e = (i, j) = i * cap + q: the entry of i in row j (the
// list is symmetric).  Sets *flags |= 4 if some reverse entry is missing.
hipError_t launch_reverse_map(const int *ell, int cap, const int *row_count, int n, int *rv, int *flags,
                              hipStream_t s);
constexpr int kMaxRow = 256;    // longest neighbour row the build supports

// Exclusive scan of n int32 values; out[n] receives the total.  tmp must hold
// scan_tmp_size(n) ints.  Also writes the maximum input to *max_out when
// max_out is not null.
size_t scan_tmp_size(int n);
hipError_t launch_exclusive_scan(const int *in, int *out, int n, int *tmp, int *max_out,
                                 hipStream_t s);

}  // namespace tsf
