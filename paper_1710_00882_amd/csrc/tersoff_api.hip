// Host runtime and C ABI of libtersoff.so (declarations and contracts in
// include/tersoff.h).  The context owns every device buffer; positions,
// types and the neighbour list stay resident between calls.
#include "internal.h"
#include "serve.h"

#include "tersoff.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace tsf;

namespace {

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t count)
    {
        if (count <= cap && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(count, 1);
        hipError_t e = hipMalloc((void **)&p, want * sizeof(T));
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

}  // namespace

struct tersoff_ctx {
    int device = 0;
    int ntypes = 0;
    std::vector<double> params;
    double max_cut = 0.0;
    DeviceTable tab{};
    void *d_table = nullptr;

    // system of the last build
    int n = 0;
    double box[3] = {0, 0, 0};
    double cutoff = 0.0, skin = 0.0;
    bool built = false;
    long long S = 0;
    int ell_cap = 32;        // row capacity for the next build (multiple of 8)
    int list_cap = 0;        // row stride of the resident list
    int max_row = 0;         // longest row of the resident list
    int atoms_per_batch = 32;
    bool batch_atoms_set = false;   // tersoff_set_batch_atoms was called (else chosen by the build)
    int force_sum = 0;              // 0: force planes + gather; 1: FP64 atomic scatter (tersoff_set_force_sum)
    int mapping = 0;                // 0: lane per packed pair; 1: lane per triplet (tersoff_set_mapping)
    int packing = 0;                // 0: separate packing kernel; 1: fused into the compute kernel where rows allow
    bool fused_ok = false;          // the resident list supports the fused packing (rows <= kFusedRowCap)
    bool rev_ready = false;         // rev holds the reverse row positions of the resident list
    bool cell_order = false;        // the caller's order is incoherent in space: atoms renumbered in the
                                    // build's cell order (perm_s, ell_s, row_count_s, types_s, pos_build_s)
    int grid[kNumPrec][4] = {};   // [precision] x {pack, compute, fixup, fused compute}

    DevBuf<double> pos_build;
    DevBuf<int> types, offsets, pcount, drop_list, jn;   // jn: compact list (S entries)
    DevBuf<int> kept;   // kept-neighbour lists: n x kKeptFast, then n x kRecCap
    DevBuf<unsigned char> recs;
    DevBuf<double> own, planes;
    DevBuf<int> cell_of, rank, cell_count, cell_start, cell_atoms, slot_cell;
    DevBuf<double> cell_pos;
    DevBuf<float4> cell_posf;
    DevBuf<int> long_rows;
    DevBuf<int> ell, row_count, scan_tmp, misc;   // misc: [0] flags, [1] max row, [2] check flags
    DevBuf<int> ell_s, row_count_s, types_s, slot_of;   // the list in the internal numbering (cell_order)
    DevBuf<int> perm_s;                                 // atom of each slot of the internal numbering
    DevBuf<double> pos_build_s;                         // positions of the build in that numbering
    DevBuf<double> pos_s;                               // positions in the internal numbering (per evaluation)
    DevBuf<unsigned char> rev;                     // reverse row positions (fused packing)
    DevBuf<unsigned long long> kmask;              // kept row positions per atom (fused packing)
    DevBuf<double> partials, force_scratch;
    DevBuf<long long> counters, counts;
    int *host_misc = nullptr;   // pinned: the build's status words, copied back without staging

    // profiling: event pairs recorded around compute / build launches
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_compute, ev_build, ev_gather, ev_pack;
    std::vector<hipEvent_t> ev_pool;

    tsf::Server *server = nullptr;   // serving runtime (tersoff_serve_start .. tersoff_serve_stop)

    // molecular-dynamics driver: per-type masses, displacement flag, energies
    DevBuf<double> md_mass, md_inv_mass, md_ev, md_partials;
    DevBuf<int> md_flag;

    std::string last_error;
};

namespace {

int fail(tersoff_ctx *c, int status, const std::string &msg)
{
    if (c) c->last_error = msg;
    return status;
}

#define HIP_TRY(ctx, expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            return fail(ctx, e_ == hipErrorOutOfMemory ? TERSOFF_E_NOMEM : TERSOFF_E_DEVICE, \
                        std::string(#expr) + ": " + hipGetErrorString(e_));            \
        }                                                                               \
    } while (0)

template <typename real>
ParamR<real> derive(const double *p)
{
    ParamR<real> r{};
    double R = p[TERSOFF_P_R], D = p[TERSOFF_P_DC], c = p[TERSOFF_P_C], d = p[TERSOFF_P_D];
    double m = p[TERSOFF_P_M], l3 = p[TERSOFF_P_LAMBDA3];
    r.A = (real)p[TERSOFF_P_A];
    r.B = (real)p[TERSOFF_P_B];
    r.lam1 = (real)p[TERSOFF_P_LAMBDA1];
    r.lam2 = (real)p[TERSOFF_P_LAMBDA2];
    r.lam3 = (real)l3;
    r.lam3m = (real)(m == 3.0 ? l3 * l3 * l3 : l3);
    r.c2d2 = (real)(p[TERSOFF_P_GAMMA] * c * c / (d * d));
    r.d2 = (real)(d * d);
    r.two_c2 = (real)(2.0 * p[TERSOFF_P_GAMMA] * c * c);
    r.h = (real)p[TERSOFF_P_H];
    r.gamma = (real)p[TERSOFF_P_GAMMA];
    r.Rc = (real)(R + D);
    r.Rin = (real)(R - D);
    r.qpi_D = (real)(M_PI / (4.0 * D));
    r.m = (real)m;
    const double lnA = std::log(p[TERSOFF_P_A]), lnB = std::log(p[TERSOFF_P_B]);
    r.lnA = (real)lnA;
    r.lnA_lo = (real)(lnA - (double)r.lnA);
    r.lam1_lo = (real)(p[TERSOFF_P_LAMBDA1] - (double)r.lam1);
    r.lnB = (real)lnB;
    r.lnB_lo = (real)(lnB - (double)r.lnB);
    r.lam2_lo = (real)(p[TERSOFF_P_LAMBDA2] - (double)r.lam2);
    r.Rc_lo = (real)((R + D) - (double)r.Rc);
    r.qpi_D_lo = (real)(M_PI / (4.0 * D) - (double)r.qpi_D);
    r.beta = (real)p[TERSOFF_P_BETA];
    return r;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

hipError_t take_event(tersoff_ctx *c, hipEvent_t *e)
{
    if (!c->ev_pool.empty()) {
        *e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

int check_compute_args(tersoff_ctx *c, const double *pos, int32_t precision, const double *energy_virial)
{
    if (!c) return TERSOFF_E_INVALID;
    if (!c->built) return fail(c, TERSOFF_E_STATE, "compute before build_neighbors");
    if (!pos || !energy_virial) return fail(c, TERSOFF_E_INVALID, "null pointer");
    if (precision != TERSOFF_FP64 && precision != TERSOFF_MIXED && precision != TERSOFF_SINGLE)
        return fail(c, TERSOFF_E_INVALID, "precision must be TERSOFF_FP64, TERSOFF_MIXED or TERSOFF_SINGLE");
    if (c->mapping == 1 && (precision == TERSOFF_SINGLE || c->force_sum == 1))
        return fail(c, TERSOFF_E_INVALID, "the lane-per-triplet mapping runs TERSOFF_FP64 and TERSOFF_MIXED "
                                          "with the force planes");
    return TERSOFF_OK;
}

// Records of one evaluation: kRecCap per atom of every (padded) batch.
size_t record_slots(const tersoff_ctx *c)
{
    const size_t nbat = ((size_t)c->n + c->atoms_per_batch - 1) / c->atoms_per_batch;
    return (size_t)kRecCap * nbat * c->atoms_per_batch;
}

// Device buffers one evaluation writes and reads back (beyond the inputs,
// the outputs and the resident neighbour list).
struct EvalBuffers {
    void *recs;          // record_region_bytes(prec, record_slots(c))
    double *planes;      // 3 kRecCap n (3 list_cap n with kmask)
    double *own;         // 3 n
    int *pcount;         // n
    int *kept;           // (kKeptFast + kRecCap) n
    int *drop_list;      // n
    double *partials;    // 8 x compute grid
    long long *counters; // 2 x compute grid
    unsigned long long *kmask;   // n, or null: no fused packing (records, kept lists, pcount used instead)
    double *pos_s;       // 3 n: positions in the internal numbering (used when cell_order)
};

// Packing, compute, dropped-atom fixup and force gather of one evaluation on
// stream s (no synchronisation, no allocation when profile is false).
int launch_evaluation(tersoff_ctx *c, const double *pos, int prec, double *energy_virial, double *f, hipStream_t s,
                      const EvalBuffers &b, bool profile)
{
    const int *grid = c->grid[prec];
    // internal numbering: when the caller's order is incoherent in space,
    // every atom is named by its slot in the build's cell order -- positions
    // permuted in, the build's renumbered rows, types and positions
    // (pos_build_s), forces stored back at the caller's indices by the gather
    // (the atomic scatter: summed in cell order, then moved) -- so that the
    // atoms of a batch, their neighbours, kept lists and force planes lie
    // together in memory.  An order that already is coherent, such as a
    // lattice's, is kept: it packs a batch more tightly than the cell
    // order's lines of cells.
    const bool slots = c->cell_order;
    const int *perm = slots ? c->perm_s.p : nullptr;
    const int *types = slots ? c->types_s.p : c->types.p;
    const int *ell = slots ? c->ell_s.p : c->ell.p;
    const int *row_count = slots ? c->row_count_s.p : c->row_count.p;
    const double *pos_build = slots ? c->pos_build_s.p : c->pos_build.p;
    PackLaunch pk{};
    pk.pos = slots ? b.pos_s : pos;
    pk.types = types;
    pk.row_count = row_count;
    pk.ell = ell;
    pk.cap = c->list_cap;
    pk.n = c->n;
    for (int d = 0; d < 3; ++d) {
        pk.L[d] = c->box[d];
        pk.invL[d] = 1.0 / c->box[d];
    }
    pk.recs = b.recs;
    pk.rlo = rlo_of(b.recs, prec, record_slots(c));
    pk.pcount = b.pcount;
    pk.kept = b.kept;
    pk.kept_more = b.kept + (size_t)kKeptFast * c->n;
    pk.own = b.own;
    pk.flags = c->misc.p;
    pk.drop_list = b.drop_list;
    pk.drop_count = c->misc.p + 3;
    pk.pos_build = pos_build;
    pk.stale_sq = 0.25 * c->skin * c->skin;
    pk.atoms_per_batch = c->atoms_per_batch;

    ComputeLaunch a{};
    a.types = types;
    a.recs = b.recs;
    a.rlo = pk.rlo;
    a.pcount = b.pcount;
    a.kept = b.kept;
    a.n = c->n;
    a.own = b.own;
    a.planes = b.planes;
    a.partials = b.partials;
    a.counters = b.counters;
    a.atoms_per_batch = c->atoms_per_batch;
    a.plane_stride = c->n;

    // fused packing: the compute kernel packs the rows itself (no records,
    // kept lists or counts in memory); planes indexed by row position
    const bool fused = b.kmask && c->fused_ok && c->packing == 1 && c->mapping == 0 && c->force_sum == 0;
    if (fused) {
        if (!c->rev_ready) {
            HIP_TRY(c, launch_reverse_index(ell, row_count, c->list_cap, c->n, c->rev.p, c->misc.p, s));
            c->rev_ready = true;
        }
        a.rows = ell;
        a.rev = c->rev.p;
        a.row_count = row_count;
        a.cap = c->list_cap;
        a.pos = pk.pos;
        a.pos_build = pos_build;
        for (int d = 0; d < 3; ++d) {
            a.L[d] = pk.L[d];
            a.invL[d] = pk.invL[d];
        }
        a.stale_sq = pk.stale_sq;
        a.flags = c->misc.p;
        a.kmask = b.kmask;
    }

    // atomic scatter (comparison point): forces summed with FP64 atomics
    // into the zeroed output (in the internal numbering: into the unused
    // plane buffer, then moved to the caller's indices); no planes, no
    // gather, only the partial sums
    const bool atomic = c->force_sum == 1;
    if (atomic) a.forces_atomic = slots ? b.planes : f;

    // event pairs (profiling only): pack (with the zeroing of the forces in
    // the atomic scatter; none with the fused packing), main kernel, fixup +
    // gather (or the partial sums)
    hipEvent_t ev[6] = {};
    if (profile)
        for (int q = fused ? 2 : 0; q < 6; ++q) HIP_TRY(c, take_event(c, &ev[q]));
    if (ev[0]) HIP_TRY(c, hipEventRecord(ev[0], s));
    if (slots) HIP_TRY(c, launch_permute_pos(pos, perm, c->n, b.pos_s, s));
    if (atomic) HIP_TRY(c, launch_fill_zero(a.forces_atomic, 3 * (size_t)c->n, s));
    if (!fused) HIP_TRY(c, launch_pack(pk, c->tab, prec, grid[0], s));
    if (ev[1]) HIP_TRY(c, hipEventRecord(ev[1], s));
    if (ev[2]) HIP_TRY(c, hipEventRecord(ev[2], s));
    int compute_grid = fused ? grid[3] : grid[1];
    if (c->mapping == 1) HIP_TRY(c, launch_compute_triplet(a, c->tab, prec, grid[1], s, &compute_grid));
    else HIP_TRY(c, launch_compute(a, c->tab, prec, compute_grid, s));
    if (ev[3]) HIP_TRY(c, hipEventRecord(ev[3], s));
    if (ev[4]) HIP_TRY(c, hipEventRecord(ev[4], s));
    const FinalizeArgs fin{b.partials, b.counters, compute_grid, energy_virial, c->counts.p, c->misc.p};
    if (fused) {
        HIP_TRY(c, launch_gather_rows(b.kmask, prec, b.planes, b.own, c->n, c->n, f, perm, fin, s));
    } else if (atomic) {
        // the partial sums alone (no rows to gather); resets the dropped count
        HIP_TRY(c, launch_gather_forces(b.pcount, prec, b.planes, b.own, 0, nullptr, c->n, f, nullptr, c->misc.p + 3,
                                        fin, s));
        if (slots) HIP_TRY(c, launch_unpermute3(b.planes, perm, c->n, f, s));
    } else {
        // an atom is dropped only with more kept neighbours than its records
        // hold, and its kept neighbours are part of its row
        if (c->max_row > kRecCap)
            HIP_TRY(c, launch_fixup_dropped(ell, c->list_cap, row_count, b.kept, pk.kept_more, b.drop_list,
                                            c->misc.p + 3, c->n, prec, b.planes, s));
        HIP_TRY(c, launch_gather_forces(b.pcount, prec, b.planes, b.own, c->n, nullptr, c->n, f, perm,
                                        c->misc.p + 3, fin, s));
    }
    if (ev[5]) HIP_TRY(c, hipEventRecord(ev[5], s));
    if (profile) {
        if (!fused) c->ev_pack.emplace_back(ev[0], ev[1]);
        c->ev_compute.emplace_back(ev[2], ev[3]);
        c->ev_gather.emplace_back(ev[4], ev[5]);
    }
    return TERSOFF_OK;
}

}  // namespace

// ---- The evaluation without allocation ----------------------------------
//
// tersoff_compute_static runs the kernels of tersoff_compute with every
// per-evaluation buffer (records, force planes, per-atom forces and counts,
// kept-neighbour lists, dropped-atom list, per-workgroup partial sums) taken
// from one file-scope device array, for builds of at most
// TERSOFF_STATIC_MAX_ATOMS atoms.  Every GPU the library runs on holds its own
// copy of the array until the process ends; host code reaches it only through
// the address hipGetSymbolAddress returns on that device.
namespace {
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kStaticAtoms = TERSOFF_STATIC_MAX_ATOMS;
constexpr size_t kStaticGrid = 8192;   // compute workgroups: at most one per batch of atoms
// records of padded batches (fewer than kWave padding atoms), at the largest
// record size (32 bytes, FP64) -- above the 20 bytes per float record
constexpr size_t kStaticRecBytes = align256((size_t)kRecCap * (kStaticAtoms + kWave) * 32);
constexpr size_t kStaticPlaneBytes = align256(3 * (size_t)kRecCap * kStaticAtoms * sizeof(double));
constexpr size_t kStaticOwnBytes = align256(3 * kStaticAtoms * sizeof(double));
constexpr size_t kStaticIntBytes = align256(kStaticAtoms * sizeof(int));
constexpr size_t kStaticKeptBytes = align256((size_t)(kKeptFast + kRecCap) * kStaticAtoms * sizeof(int));
constexpr size_t kStaticPartialBytes = align256(8 * kStaticGrid * sizeof(double));
constexpr size_t kStaticCounterBytes = align256(2 * kStaticGrid * sizeof(long long));
constexpr size_t kStaticBytes = kStaticRecBytes + kStaticPlaneBytes + 3 * kStaticOwnBytes + 2 * kStaticIntBytes +
                                kStaticKeptBytes + kStaticPartialBytes + kStaticCounterBytes;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// The address of `scratch` on device dev (current), looked up once per device.
hipError_t static_scratch(int dev, unsigned char **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

extern "C" {

const char *tersoff_strerror(int status)
{
    switch (status) {
    case TERSOFF_OK: return "ok";
    case TERSOFF_E_INVALID: return "invalid argument";
    case TERSOFF_E_NOMEM: return "out of device memory";
    case TERSOFF_E_BOX: return "box shorter than twice the list radius";
    case TERSOFF_E_OVERFLOW: return "neighbour capacity exceeded";
    case TERSOFF_E_STALE: return "neighbour list is stale (an atom moved more than skin/2)";
    case TERSOFF_E_DEVICE: return "HIP runtime error";
    case TERSOFF_E_AGAIN: return "no slot or memory free";
    case TERSOFF_E_PENDING: return "result not ready";
    case TERSOFF_E_STATE: return "call out of order";
    default: return "unknown status";
    }
}

const char *tersoff_last_error(const tersoff_ctx *ctx)
{
    return ctx ? ctx->last_error.c_str() : "";
}

int tersoff_create(const double *params, int32_t ntypes, tersoff_ctx **out)
{
    if (!out) return TERSOFF_E_INVALID;
    *out = nullptr;
    if (!params || ntypes < 1 || ntypes > TERSOFF_MAX_TYPES) return TERSOFF_E_INVALID;
    const int ne = ntypes * ntypes * ntypes;
    for (int e = 0; e < ne; ++e) {
        const double *p = params + (size_t)e * TERSOFF_NPARAM;
        for (int f = 0; f < TERSOFF_NPARAM; ++f)
            if (!std::isfinite(p[f])) return TERSOFF_E_INVALID;
        if (!(p[TERSOFF_P_A] > 0) || !(p[TERSOFF_P_B] > 0) ||
            !(p[TERSOFF_P_DC] > 0) || !(p[TERSOFF_P_R] - p[TERSOFF_P_DC] >= 0) ||
            !(p[TERSOFF_P_ETA] > 0) || !(p[TERSOFF_P_BETA] >= 0) || p[TERSOFF_P_C] == 0 ||
            p[TERSOFF_P_D] == 0 || !(p[TERSOFF_P_M] == 1.0 || p[TERSOFF_P_M] == 3.0))
            return TERSOFF_E_INVALID;
    }
    tersoff_ctx *c = new (std::nothrow) tersoff_ctx();
    if (!c) return TERSOFF_E_NOMEM;
    (void)hipGetDevice(&c->device);
    c->ntypes = ntypes;
    c->params.assign(params, params + (size_t)ne * TERSOFF_NPARAM);

    std::vector<ParamR<float>> pf(ne);
    std::vector<ParamR<double>> pd(ne);
    std::vector<ParamX> px(ne);
    std::vector<double> packsq((size_t)ntypes * ntypes, 0.0);
    for (int e = 0; e < ne; ++e) {
        const double *p = params + (size_t)e * TERSOFF_NPARAM;
        pf[e] = derive<float>(p);
        pd[e] = derive<double>(p);
        double cut = p[TERSOFF_P_R] + p[TERSOFF_P_DC];
        px[e].cutsq = cut * cut;
        px[e].logbeta = p[TERSOFF_P_BETA] > 0 ? std::log(p[TERSOFF_P_BETA]) : -INFINITY;
        px[e].eta = p[TERSOFF_P_ETA];
        px[e].inv2eta = 1.0 / (2.0 * p[TERSOFF_P_ETA]);
        px[e].A = p[TERSOFF_P_A];
        px[e].B = p[TERSOFF_P_B];
        px[e].lam1 = p[TERSOFF_P_LAMBDA1];
        px[e].lam2 = p[TERSOFF_P_LAMBDA2];
        c->max_cut = std::max(c->max_cut, cut);
    }
    // packing radius of neighbour n of centre i: every entry (ti, *, tn)
    // (n as the bond partner or as a third atom), made symmetric in (ti, tn)
    // so that i packs n exactly when n packs i
    for (int ti = 0; ti < ntypes; ++ti)
        for (int tj = 0; tj < ntypes; ++tj)
            for (int tk = 0; tk < ntypes; ++tk) {
                double cs = px[(ti * ntypes + tj) * ntypes + tk].cutsq;
                double &a = packsq[(size_t)ti * ntypes + tk];
                double &b = packsq[(size_t)tk * ntypes + ti];
                a = std::max(a, cs);
                b = std::max(b, cs);
            }
    size_t off_pf = 0;
    size_t off_pd = off_pf + ((sizeof(ParamR<float>) * ne + 255) / 256) * 256;
    size_t off_px = off_pd + ((sizeof(ParamR<double>) * ne + 255) / 256) * 256;
    size_t off_pk = off_px + ((sizeof(ParamX) * ne + 255) / 256) * 256;
    size_t total = off_pk + sizeof(double) * packsq.size();
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data() + off_pf, pf.data(), sizeof(ParamR<float>) * ne);
    std::memcpy(host.data() + off_pd, pd.data(), sizeof(ParamR<double>) * ne);
    std::memcpy(host.data() + off_px, px.data(), sizeof(ParamX) * ne);
    std::memcpy(host.data() + off_pk, packsq.data(), sizeof(double) * packsq.size());
    hipError_t e = hipMalloc(&c->d_table, total);
    if (e == hipSuccess) e = hipMemcpy(c->d_table, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        int st = e == hipErrorOutOfMemory ? TERSOFF_E_NOMEM : TERSOFF_E_DEVICE;
        if (c->d_table) (void)hipFree(c->d_table);
        delete c;
        return st;
    }
    unsigned char *base = static_cast<unsigned char *>(c->d_table);
    c->tab.ntypes = ntypes;
    c->tab.pf = reinterpret_cast<const ParamR<float> *>(base + off_pf);
    c->tab.pd = reinterpret_cast<const ParamR<double> *>(base + off_pd);
    c->tab.px = reinterpret_cast<const ParamX *>(base + off_px);
    c->tab.packsq = reinterpret_cast<const double *>(base + off_pk);
    c->tab.lam3_zero = ntypes == 1 && params[TERSOFF_P_LAMBDA3] == 0.0;
    // g(theta) and the exponential factor of triplet (i; j, k) equal those of
    // (i; k, j) when these parameters agree (the compute kernel then forms
    // both roles of a triplet from one evaluation)
    c->tab.sym3 = 1;
    for (int ti = 0; ti < ntypes; ++ti)
        for (int tj = 0; tj < ntypes; ++tj)
            for (int tk = 0; tk < ntypes; ++tk) {
                const double *p = params + (size_t)((ti * ntypes + tj) * ntypes + tk) * TERSOFF_NPARAM;
                const double *q = params + (size_t)((ti * ntypes + tk) * ntypes + tj) * TERSOFF_NPARAM;
                for (int f : {TERSOFF_P_C, TERSOFF_P_D, TERSOFF_P_H, TERSOFF_P_GAMMA, TERSOFF_P_LAMBDA3, TERSOFF_P_M})
                    if (p[f] != q[f]) c->tab.sym3 = 0;
            }
    *out = c;
    return TERSOFF_OK;
}

void tersoff_destroy(tersoff_ctx *c)
{
    if (!c) return;
    tsf::server_destroy(c->server);
    c->server = nullptr;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->pos_build.release(); c->types.release(); c->offsets.release(); c->jn.release();
    c->kept.release(); c->own.release(); c->planes.release(); c->rev.release(); c->kmask.release();
    c->ell_s.release(); c->row_count_s.release(); c->types_s.release(); c->slot_of.release(); c->pos_s.release();
    c->perm_s.release(); c->pos_build_s.release();
    c->pcount.release(); c->drop_list.release(); c->recs.release();
    c->cell_of.release(); c->rank.release(); c->cell_count.release(); c->cell_start.release();
    c->cell_atoms.release(); c->slot_cell.release(); c->cell_pos.release(); c->ell.release(); c->row_count.release();
    c->cell_posf.release(); c->long_rows.release();
    c->scan_tmp.release(); c->misc.release(); c->partials.release(); c->force_scratch.release();
    c->counters.release(); c->counts.release();
    c->md_mass.release(); c->md_inv_mass.release(); c->md_ev.release(); c->md_partials.release();
    c->md_flag.release();
    for (auto &pr : c->ev_compute) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto &pr : c->ev_build) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto &pr : c->ev_gather) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto &pr : c->ev_pack) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->d_table) (void)hipFree(c->d_table);
    if (c->host_misc) (void)hipHostFree(c->host_misc);
    delete c;
}

int tersoff_profile(tersoff_ctx *c, int32_t enable)
{
    if (!c) return TERSOFF_E_INVALID;
    c->profiling = enable != 0;
    return TERSOFF_OK;
}

int tersoff_profile_read(tersoff_ctx *c, double out[8])
{
    if (!c || !out) return TERSOFF_E_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    std::vector<std::pair<hipEvent_t, hipEvent_t>> *lists[4] = {&c->ev_compute, &c->ev_build, &c->ev_gather,
                                                                &c->ev_pack};
    for (int l = 0; l < 4; ++l) {
        double t = 0.0;
        for (auto &pr : *lists[l]) {
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, pr.first, pr.second));
            t += ms;
        }
        const int slot = 2 * l;
        out[slot] = t;
        out[slot + 1] = (double)lists[l]->size();
        for (auto &pr : *lists[l]) { c->ev_pool.push_back(pr.first); c->ev_pool.push_back(pr.second); }
        lists[l]->clear();
    }
    return TERSOFF_OK;
}

int tersoff_set_batch_atoms(tersoff_ctx *c, int32_t atoms)
{
    if (!c) return TERSOFF_E_INVALID;
    if (atoms < 1 || atoms > kWave) return fail(c, TERSOFF_E_INVALID, "batch atoms must be in [1, 64]");
    c->atoms_per_batch = atoms;
    c->batch_atoms_set = true;
    if (c->built) {
        int gmax = 0;
        for (int pr = 0; pr < kNumPrec; ++pr) {
            compute_grids(pr, c->tab, false, c->n, atoms, c->grid[pr]);
            gmax = std::max({gmax, c->grid[pr][1], c->grid[pr][3]});
        }
        HIP_TRY(c, c->partials.ensure(8 * (size_t)gmax));
        HIP_TRY(c, c->counters.ensure(2 * (size_t)gmax));
    }
    return TERSOFF_OK;
}

int tersoff_set_force_sum(tersoff_ctx *c, int32_t mode)
{
    if (!c) return TERSOFF_E_INVALID;
    if (mode != 0 && mode != 1) return fail(c, TERSOFF_E_INVALID, "force-sum mode must be 0 or 1");
    c->force_sum = mode;
    return TERSOFF_OK;
}

int tersoff_set_packing(tersoff_ctx *c, int32_t mode)
{
    if (!c) return TERSOFF_E_INVALID;
    if (mode != 0 && mode != 1) return fail(c, TERSOFF_E_INVALID, "packing mode must be 0 or 1");
    c->packing = mode;
    return TERSOFF_OK;
}

int tersoff_set_mapping(tersoff_ctx *c, int32_t mode)
{
    if (!c) return TERSOFF_E_INVALID;
    if (mode != 0 && mode != 1) return fail(c, TERSOFF_E_INVALID, "mapping must be 0 or 1");
    c->mapping = mode;
    return TERSOFF_OK;
}

int64_t tersoff_num_atoms(const tersoff_ctx *c)
{
    return (c && c->built) ? c->n : 0;
}

int tersoff_build_neighbors(tersoff_ctx *c, const double *pos, const int32_t *types, int64_t n,
                            const double box[3], double cutoff, double skin, void *stream)
{
    if (!c) return TERSOFF_E_INVALID;
    c->last_error.clear();
    if (!pos || !types || !box) return fail(c, TERSOFF_E_INVALID, "null pointer");
    if (n < 1 || n > (int64_t)(1 << 24)) return fail(c, TERSOFF_E_INVALID, "n must be in [1, 2^24]");
    if (!(cutoff >= c->max_cut * (1.0 - 1e-12)) || !std::isfinite(cutoff))
        return fail(c, TERSOFF_E_INVALID, "cutoff below the largest R + D of the table");
    if (!(skin >= 0) || !std::isfinite(skin)) return fail(c, TERSOFF_E_INVALID, "skin must be >= 0");
    const double rc = cutoff + skin;
    for (int a = 0; a < 3; ++a) {
        if (!(box[a] > 0) || !std::isfinite(box[a])) return fail(c, TERSOFF_E_INVALID, "box must be positive");
        if (box[a] < 2.0 * rc) return fail(c, TERSOFF_E_BOX, "box length below 2 (cutoff + skin)");
    }
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = as_stream(stream);
    const int N = (int)n;
    c->built = false;

    hipEvent_t evb0 = nullptr, evb1 = nullptr;
    if (c->profiling) {
        HIP_TRY(c, take_event(c, &evb0));
        HIP_TRY(c, take_event(c, &evb1));
        HIP_TRY(c, hipEventRecord(evb0, s));
    }
    CellGrid g{};
    long long ncell = 1;
    for (int a = 0; a < 3; ++a) {
        g.L[a] = box[a];
        g.invL[a] = 1.0 / box[a];
        g.Lf[a] = (float)box[a];
        g.invLf[a] = (float)(1.0 / box[a]);
        g.nc[a] = std::max(1, (int)std::floor(box[a] / (rc * (1.0 + 1e-10))));
        g.nc[a] = std::min(g.nc[a], 1024);
        g.cell_w[a] = box[a] / g.nc[a];
        ncell *= g.nc[a];
    }
    g.Lsum = g.Lf[0] + g.Lf[1] + g.Lf[2];
    HIP_TRY(c, c->misc.ensure(8));
    HIP_TRY(c, c->cell_of.ensure(N));
    HIP_TRY(c, c->rank.ensure(N));
    HIP_TRY(c, c->cell_count.ensure(ncell));
    HIP_TRY(c, c->cell_start.ensure(ncell + 1));
    HIP_TRY(c, c->cell_atoms.ensure(N));
    HIP_TRY(c, c->slot_cell.ensure(N));
    HIP_TRY(c, c->cell_pos.ensure(3 * (size_t)N));
    HIP_TRY(c, c->cell_posf.ensure((size_t)N + kPosPad));
    HIP_TRY(c, c->long_rows.ensure((size_t)N));
    HIP_TRY(c, c->row_count.ensure(N));
    HIP_TRY(c, c->pcount.ensure(N));
    HIP_TRY(c, c->kept.ensure((size_t)(kKeptFast + kRecCap) * N));
    HIP_TRY(c, c->drop_list.ensure(N));
    HIP_TRY(c, c->offsets.ensure((size_t)N + 1));
    HIP_TRY(c, c->scan_tmp.ensure(std::max(scan_tmp_size((int)ncell), scan_tmp_size(N))));
    HIP_TRY(c, c->pos_build.ensure(3 * (size_t)N));
    HIP_TRY(c, c->types.ensure(N));

    // misc: [0] compute flags, [1] longest row, [2] build flags, [3] dropped
    // count, [4] rows left to the long-row search, [6] consecutive atoms in
    // the same or adjacent cells.  One host
    // synchronisation at the end: a row longer than the capacity of the
    // attempt (known only from the scan) repeats it with the needed one.
    // The evaluation reads the row buffer itself (row i at i * cap); the
    // compact list is formed only when asked for (tersoff_get_neighbors).
    HIP_TRY(c, hipMemsetAsync(c->misc.p, 0, 8 * sizeof(int), s));
    HIP_TRY(c, hipMemsetAsync(c->cell_count.p, 0, sizeof(int) * ncell, s));
    HIP_TRY(c, launch_bin_atoms(pos, types, N, c->ntypes, g, c->cell_of.p, c->rank.p, c->cell_count.p,
                                c->misc.p + 2, c->types.p, c->misc.p + 6, s));
    HIP_TRY(c, launch_exclusive_scan(c->cell_count.p, c->cell_start.p, (int)ncell, c->scan_tmp.p, nullptr, s));
    ScatterLaunch sca{};
    sca.pos = pos;
    sca.n = N;
    sca.cell_of = c->cell_of.p;
    sca.rank = c->rank.p;
    sca.cell_start = c->cell_start.p;
    sca.cell_atoms = c->cell_atoms.p;
    sca.cell_pos = c->cell_pos.p;
    sca.cell_posf = c->cell_posf.p;
    sca.pos_copy = c->pos_build.p;
    sca.slot_cell = c->slot_cell.p;
    sca.g = g;
    HIP_TRY(c, launch_scatter_cells(sca, 0, s));
    SearchLaunch sl{};
    sl.g = g;
    sl.n = N;
    sl.rc2 = rc * rc;
    sl.rcs = (float)rc;
    sl.cell_start = c->cell_start.p;
    sl.cell_count = c->cell_count.p;
    sl.cell_atoms = c->cell_atoms.p;
    sl.cell_of = c->cell_of.p;
    sl.slot_cell = c->slot_cell.p;
    sl.cell_pos = c->cell_pos.p;
    sl.cell_posf = c->cell_posf.p;
    sl.row_count = c->row_count.p;
    sl.long_rows = c->long_rows.p;
    sl.n_long = c->misc.p + 4;
    HIP_TRY(c, c->own.ensure(3 * (size_t)N));
    if (!c->host_misc) HIP_TRY(c, hipHostMalloc((void **)&c->host_misc, 16 * sizeof(int), hipHostMallocDefault));
    HIP_TRY(c, c->counts.ensure(2));
    HIP_TRY(c, hipMemsetAsync(c->counts.p, 0, 2 * sizeof(long long), s));
    int host[8] = {};
    for (int attempt = 0; attempt < 2; ++attempt) {
        if ((long long)N * c->ell_cap >= (1LL << 31)) return fail(c, TERSOFF_E_INVALID, "n x row capacity >= 2^31");
        const size_t cap_entries = (size_t)N * c->ell_cap;
        HIP_TRY(c, c->ell.ensure(cap_entries));
        if (attempt > 0) HIP_TRY(c, hipMemsetAsync(c->misc.p + 4, 0, sizeof(int), s));
        sl.cap = c->ell_cap;
        sl.ell = c->ell.p;
        HIP_TRY(c, launch_search(sl, 0, s));
        HIP_TRY(c, launch_exclusive_scan(c->row_count.p, c->offsets.p, N, c->scan_tmp.p, c->misc.p + 1, s));
        HIP_TRY(c, hipMemcpyAsync(c->host_misc, c->misc.p, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipMemcpyAsync(c->host_misc + 5, c->offsets.p + N, sizeof(int), hipMemcpyDeviceToHost, s));
        if (evb1) HIP_TRY(c, hipEventRecord(evb1, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        std::copy(c->host_misc, c->host_misc + 8, host);
        if (host[2] & 1) return fail(c, TERSOFF_E_INVALID, "non-finite position");
        if (host[2] & 2) return fail(c, TERSOFF_E_INVALID, "type out of range");
        if (host[1] <= c->ell_cap) break;
        if (host[1] > kMaxRow) return fail(c, TERSOFF_E_OVERFLOW, "an atom has more than 256 neighbours in range");
        c->ell_cap = ((host[1] + 7) / 8) * 8;   // repeat once with the needed capacity
    }
    if (evb1) c->ev_build.emplace_back(evb0, evb1);
    if (host[1] > c->ell_cap) return fail(c, TERSOFF_E_OVERFLOW, "row capacity retry failed");
    c->list_cap = c->ell_cap;
    c->max_row = host[1];
    if (host[5] < 0) return fail(c, TERSOFF_E_INVALID, "list longer than 2^31 entries");
    c->S = host[5];
    // the next build starts from the capacity this list needed (plus a margin)
    c->ell_cap = std::max(8, ((host[1] + 2 + 7) / 8) * 8);

    // the fused packing (a comparison point) needs each entry's position in
    // its neighbour's row; formed by the first fused evaluation of this list
    c->fused_ok = c->list_cap <= kFusedRowCap;
    c->rev_ready = false;
    // the caller's order is kept when at least half of its consecutive atoms
    // (the pairs i, i + 1 with i mod 64 != 63 that the binning examines) share
    // or neighbour a cell
    const long long examined = (long long)N - 1 - ((long long)N - 1) / 64;
    c->cell_order = 2LL * host[6] < examined;
    if (c->cell_order) {
        // the list in the internal numbering (cell-order slots)
        HIP_TRY(c, c->ell_s.ensure((size_t)N * c->list_cap));
        HIP_TRY(c, c->row_count_s.ensure(N));
        HIP_TRY(c, c->types_s.ensure(N));
        HIP_TRY(c, c->slot_of.ensure(N));
        HIP_TRY(c, c->perm_s.ensure(N));
        HIP_TRY(c, c->pos_build_s.ensure(3 * (size_t)N));
        HIP_TRY(c, launch_renumber_rows(c->ell.p, c->row_count.p, c->list_cap, c->cell_atoms.p, c->cell_start.p,
                                        c->cell_count.p, (int)ncell, c->types.p, c->pos_build.p, N, c->perm_s.p,
                                        c->slot_of.p, c->ell_s.p, c->row_count_s.p, c->types_s.p,
                                        c->pos_build_s.p, s));
    }

    c->n = N;
    for (int a = 0; a < 3; ++a) c->box[a] = box[a];
    c->cutoff = cutoff;
    c->skin = skin;
    // default batch: 32 centre atoms; 64 with several species, whose uneven
    // kept counts leave each group's last batch partly filled (fewer, larger
    // groups: 256k-atom two-species packing 40 -> 37 us, compute 77 -> 74
    // us; silicon is fastest at 32); 16 below 128k atoms, where the number of batches
    // rather than the work per batch limits the packing and compute kernels
    if (!c->batch_atoms_set) c->atoms_per_batch = N < 131072 ? 16 : (c->ntypes > 1 ? 64 : 32);
    int gmax = 0;
    for (int pr = 0; pr < kNumPrec; ++pr) {
        compute_grids(pr, c->tab, false, N, c->atoms_per_batch, c->grid[pr]);
        gmax = std::max({gmax, c->grid[pr][1], c->grid[pr][3]});
    }
    HIP_TRY(c, c->partials.ensure(8 * (size_t)gmax));
    HIP_TRY(c, c->counters.ensure(2 * (size_t)gmax));
    c->built = true;
    return TERSOFF_OK;
}

int tersoff_compute(tersoff_ctx *c, const double *pos, int32_t precision, double *energy_virial,
                    double *forces, void *stream)
{
    const int st = check_compute_args(c, pos, precision, energy_virial);
    if (st != TERSOFF_OK) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    const int prec = precision;
    double *f = forces;
    if (!f) {
        HIP_TRY(c, c->force_scratch.ensure(3 * (size_t)c->n));
        f = c->force_scratch.p;
    }
    const size_t slots = record_slots(c);
    HIP_TRY(c, c->recs.ensure(record_region_bytes(prec, slots)));
    HIP_TRY(c, c->planes.ensure(3 * (size_t)std::max(kRecCap, c->list_cap) * (size_t)c->n));
    EvalBuffers b{};
    b.recs = c->recs.p;
    b.planes = c->planes.p;
    b.own = c->own.p;
    b.pcount = c->pcount.p;
    b.kept = c->kept.p;
    b.drop_list = c->drop_list.p;
    b.partials = c->partials.p;
    b.counters = c->counters.p;
    if (c->cell_order) {
        HIP_TRY(c, c->pos_s.ensure(3 * (size_t)c->n));
        b.pos_s = c->pos_s.p;
    }
    if (c->fused_ok && c->packing == 1) {
        HIP_TRY(c, c->rev.ensure((size_t)c->n * c->list_cap));
        HIP_TRY(c, c->kmask.ensure(c->n));
        b.kmask = c->kmask.p;
    }
    return launch_evaluation(c, pos, prec, energy_virial, f, as_stream(stream), b, c->profiling);
}

int tersoff_compute_static(tersoff_ctx *c, const double *pos, int32_t precision, double *energy_virial,
                           double *forces, void *stream)
{
    const int st = check_compute_args(c, pos, precision, energy_virial);
    if (st != TERSOFF_OK) return st;
    const int prec = precision;
    if (c->n > TERSOFF_STATIC_MAX_ATOMS)
        return fail(c, TERSOFF_E_INVALID, "tersoff_compute_static: the build has more than TERSOFF_STATIC_MAX_ATOMS atoms");
    if (record_region_bytes(prec, record_slots(c)) > kStaticRecBytes || c->grid[prec][1] > (int)kStaticGrid)
        return fail(c, TERSOFF_E_INVALID, "tersoff_compute_static: batch layout beyond the static scratch");
    HIP_TRY(c, hipSetDevice(c->device));
    unsigned char *base = nullptr;
    HIP_TRY(c, static_scratch(c->device, &base));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += bytes;
        return p;
    };
    EvalBuffers b{};
    b.recs = take(kStaticRecBytes);
    b.planes = reinterpret_cast<double *>(take(kStaticPlaneBytes));
    b.own = reinterpret_cast<double *>(take(kStaticOwnBytes));
    double *force_scratch = reinterpret_cast<double *>(take(kStaticOwnBytes));
    b.pos_s = reinterpret_cast<double *>(take(kStaticOwnBytes));
    b.pcount = reinterpret_cast<int *>(take(kStaticIntBytes));
    b.drop_list = reinterpret_cast<int *>(take(kStaticIntBytes));
    b.kept = reinterpret_cast<int *>(take(kStaticKeptBytes));
    b.partials = reinterpret_cast<double *>(take(kStaticPartialBytes));
    b.counters = reinterpret_cast<long long *>(take(kStaticCounterBytes));
    return launch_evaluation(c, pos, prec, energy_virial, forces ? forces : force_scratch, as_stream(stream), b,
                             false);
}

int tersoff_check(tersoff_ctx *c, void *stream)
{
    if (!c) return TERSOFF_E_INVALID;
    if (!c->misc.p) return TERSOFF_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = as_stream(stream);
    int flags = 0;
    HIP_TRY(c, hipMemcpyAsync(&flags, c->misc.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemsetAsync(c->misc.p, 0, sizeof(int), s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (flags & kFlagOverflow) return fail(c, TERSOFF_E_OVERFLOW, "an atom exceeded the per-batch neighbour capacity");
    if (flags & kFlagStale) return fail(c, TERSOFF_E_STALE, "an atom moved more than skin/2 since the last build");
    if (flags & kFlagAsym) return fail(c, TERSOFF_E_DEVICE, "kept-neighbour sets are not symmetric");
    return TERSOFF_OK;
}

int tersoff_get_neighbors(tersoff_ctx *c, int64_t *offsets, int32_t *idx, int64_t cap, int64_t *total)
{
    if (!c) return TERSOFF_E_INVALID;
    if (!c->built) return fail(c, TERSOFF_E_STATE, "no neighbour list");
    if (!offsets || !total) return fail(c, TERSOFF_E_INVALID, "null pointer");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    std::vector<int> off((size_t)c->n + 1);
    HIP_TRY(c, hipMemcpy(off.data(), c->offsets.p, sizeof(int) * off.size(), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < off.size(); ++i) offsets[i] = off[i];
    *total = c->S;
    if (cap < c->S || (!idx && c->S > 0)) return fail(c, TERSOFF_E_INVALID, "idx capacity below list length");
    if (c->S > 0) {
        HIP_TRY(c, c->jn.ensure((size_t)c->S));
        HIP_TRY(c, launch_compact_list(c->ell.p, c->list_cap, c->row_count.p, c->offsets.p, c->n, nullptr, c->jn.p,
                                       c->S, nullptr, nullptr));
        HIP_TRY(c, hipMemcpy(idx, c->jn.p, sizeof(int) * (size_t)c->S, hipMemcpyDeviceToHost));
    }
    return TERSOFF_OK;
}

int tersoff_get_counts(tersoff_ctx *c, int64_t counts[3])
{
    if (!c || !counts) return TERSOFF_E_INVALID;
    if (!c->built) return fail(c, TERSOFF_E_STATE, "no neighbour list");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    long long h[2] = {0, 0};
    HIP_TRY(c, hipMemcpy(h, c->counts.p, sizeof(h), hipMemcpyDeviceToHost));
    counts[0] = c->S;
    counts[1] = h[0];
    counts[2] = h[1];
    return TERSOFF_OK;
}

int tersoff_serve_start(tersoff_ctx *c, const tersoff_serve_config *cfg)
{
    if (!c || !cfg) return TERSOFF_E_INVALID;
    if (c->server) return fail(c, TERSOFF_E_STATE, "serving already started");
    tsf::ServerEnv env{c->device, c->ntypes, c->max_cut, c->tab};
    std::string err;
    const int st = tsf::server_create(env, *cfg, &c->server, err);
    if (st != TERSOFF_OK) return fail(c, st, err);
    return TERSOFF_OK;
}

int tersoff_serve_stop(tersoff_ctx *c)
{
    if (!c) return TERSOFF_E_INVALID;
    if (!c->server) return fail(c, TERSOFF_E_STATE, "serving not started");
    tsf::server_destroy(c->server);
    c->server = nullptr;
    return TERSOFF_OK;
}

int tersoff_submit(tersoff_ctx *c, const tersoff_request *req, uint64_t *ticket)
{
    if (!c || !req || !ticket) return TERSOFF_E_INVALID;
    if (!c->server) return TERSOFF_E_STATE;
    std::string err;
    // messages of the thread-safe calls are not stored in the context
    return tsf::server_submit(c->server, *req, ticket, err);
}

int tersoff_poll(tersoff_ctx *c, uint64_t ticket, double timeout_ms, tersoff_result *res)
{
    if (!c || !res) return TERSOFF_E_INVALID;
    if (!c->server) return TERSOFF_E_STATE;
    std::string err;
    return tsf::server_poll(c->server, ticket, res, timeout_ms, err);
}

int tersoff_serve_stats(tersoff_ctx *c, double out[6])
{
    if (!c || !out) return TERSOFF_E_INVALID;
    if (!c->server) return fail(c, TERSOFF_E_STATE, "serving not started");
    tsf::server_stats(c->server, out);
    return TERSOFF_OK;
}

int tersoff_md_run(tersoff_ctx *c, double *pos, double *vel, double *forces, const int32_t *types, int64_t n,
                   const double box[3], const tersoff_md_config *cfg, double out[4], void *stream)
{
    if (!c) return TERSOFF_E_INVALID;
    if (!pos || !vel || !forces || !types || !box || !cfg || !out || !cfg->mass)
        return fail(c, TERSOFF_E_INVALID, "null pointer");
    if (!(cfg->dt > 0) || !std::isfinite(cfg->dt) || cfg->nsteps < 0 || !(cfg->skin > 0) || !std::isfinite(cfg->skin))
        return fail(c, TERSOFF_E_INVALID, "dt and skin must be positive, nsteps >= 0");
    if (cfg->precision < TERSOFF_FP64 || cfg->precision > TERSOFF_SINGLE)
        return fail(c, TERSOFF_E_INVALID, "unknown precision");
    std::vector<double> mass(cfg->mass, cfg->mass + c->ntypes), inv(c->ntypes);
    for (int t = 0; t < c->ntypes; ++t) {
        if (!(mass[t] > 0) || !std::isfinite(mass[t])) return fail(c, TERSOFF_E_INVALID, "masses must be positive");
        inv[t] = 1.0 / mass[t];
    }
    const double cutoff = cfg->cutoff > 0 ? cfg->cutoff : c->max_cut;
    // acceleration of 1 eV / (A amu) in A / ps^2: (1.602176634e-19 J / 1e-10 m)
    // / 1.66053906660e-27 kg, expressed in 1e14 m/s^2
    const double conv = 1.602176634e-19 / 1e-10 / 1.66053906660e-27 / 1e14;
    const int N = (int)n;
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = as_stream(stream);
    HIP_TRY(c, c->md_mass.ensure(c->ntypes));
    HIP_TRY(c, c->md_inv_mass.ensure(c->ntypes));
    HIP_TRY(c, c->md_ev.ensure(7));
    HIP_TRY(c, c->md_flag.ensure(1));
    HIP_TRY(c, c->md_partials.ensure(md_kinetic_blocks()));
    HIP_TRY(c, hipMemcpyAsync(c->md_mass.p, mass.data(), sizeof(double) * mass.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->md_inv_mass.p, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, s));

    int st = tersoff_build_neighbors(c, pos, types, n, box, cutoff, cfg->skin, stream);
    if (st != TERSOFF_OK) return st;
    int builds = 1;
    st = tersoff_compute(c, pos, cfg->precision, c->md_ev.p, forces, stream);
    if (st != TERSOFF_OK) return st;
    const double half = 0.5 * cfg->dt * conv;
    const double lim2 = 0.25 * cfg->skin * cfg->skin;
    for (int step = 0; step < cfg->nsteps; ++step) {
        HIP_TRY(c, launch_md_kick(vel, forces, types, c->md_inv_mass.p, half, N, s));
        HIP_TRY(c, launch_md_drift(pos, vel, cfg->dt, N, s));
        HIP_TRY(c, hipMemsetAsync(c->md_flag.p, 0, sizeof(int), s));
        HIP_TRY(c, launch_md_displaced(pos, c->pos_build.p, lim2, N, c->md_flag.p, s));
        int moved = 0;
        HIP_TRY(c, hipMemcpyAsync(&moved, c->md_flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        if (moved) {
            st = tersoff_build_neighbors(c, pos, types, n, box, cutoff, cfg->skin, stream);
            if (st != TERSOFF_OK) return st;
            ++builds;
        }
        st = tersoff_compute(c, pos, cfg->precision, c->md_ev.p, forces, stream);
        if (st != TERSOFF_OK) return st;
        HIP_TRY(c, launch_md_kick(vel, forces, types, c->md_inv_mass.p, half, N, s));
    }
    HIP_TRY(c, launch_md_kinetic(vel, types, c->md_mass.p, N, c->md_partials.p, s));
    std::vector<double> part(md_kinetic_blocks());
    double ev[7];
    HIP_TRY(c, hipMemcpyAsync(part.data(), c->md_partials.p, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(ev, c->md_ev.p, sizeof(ev), hipMemcpyDeviceToHost, s));
    st = tersoff_check(c, stream);   // synchronises; overflow / stale flags of the run
    if (st != TERSOFF_OK) return st;
    double mv2 = 0.0;
    for (double v : part) mv2 += v;
    const double ekin = 0.5 * mv2 / conv;
    const double kB = 8.617333262e-5;   // eV / K
    out[0] = ev[0];
    out[1] = ekin;
    out[2] = builds;
    out[3] = 2.0 * ekin / (3.0 * (double)n * kB);
    return TERSOFF_OK;
}

}  // extern "C"
