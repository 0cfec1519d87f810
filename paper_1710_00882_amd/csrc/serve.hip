// Serving runtime: many small, independent configurations (each with its own
// periodic box) evaluated in batches.
//
// Requests wait in a FIFO queue.  A worker thread forms a batch from the head
// of the queue -- as many requests as fit the batch's atom, configuration,
// and cell capacities (the device-memory budget fixed at start) and
// share one precision -- concatenates their atoms into pinned staging
// buffers, and launches it on one of two buffer sets, each with its own
// stream.  While one batch runs, the next is formed from whatever arrived in
// the meantime and launched on the other set (continuous batching); results
// are handed back in launch order.
//
// The device work of a batch is one captured HIP graph per buffer set and
// precision, replayed for every batch: the kernels read the batch's sizes and
// per-configuration descriptors from device memory, so a replay needs only
// the host-to-device copies of the inputs and descriptors before it and the
// copies of the results after it.  Graph contents: clear counters -> bin every
// configuration's atoms into its own cells -> scan -> scatter -> neighbour
// search over all configurations (rows at a fixed stride) -> pack -> energy / force /
// virial kernel (per-atom energy and virial) -> dropped-atom fixup -> force
// gather -> per-configuration reduction.  A configuration's result does not
// depend on the other configurations of its batch or on its place in it.
#include "serve.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace tsf {

namespace {

constexpr int kLanes = 2;          // buffer sets (batches in flight)
// centre atoms per batch of the packing and compute kernels (a serving batch
// holds up to 262144 atoms; 32 against 16: device-resident capacity 8.4e5 ->
// 8.8e5 configurations/s, FP64 5.3e5 -> 6.0e5)
constexpr int kServeBatchAtoms = 32;

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

template <typename T>
struct Dev {
    T *p = nullptr;
    hipError_t alloc(size_t n, size_t &total)
    {
        const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        hipError_t e = hipMalloc((void **)&p, bytes);
        if (e == hipSuccess) total += bytes;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
};

template <typename T>
struct Pinned {
    T *p = nullptr;
    hipError_t alloc(size_t n)
    {
        return hipHostMalloc((void **)&p, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault);
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
    }
};

// Host threads that share the per-request copies of a batch (staging the
// inputs into pinned memory, handing forces back) with the worker thread.
class CopyPool {
public:
    explicit CopyPool(int helpers)
    {
        for (int h = 0; h < helpers; ++h) th_.emplace_back([this] { loop(); });
    }
    ~CopyPool()
    {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    // f(k) for every k in [0, parts), spread over the helpers and the caller.
    void run(int parts, const std::function<void(int)> &f)
    {
        if (th_.empty() || parts < 2) {
            for (int k = 0; k < parts; ++k) f(k);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(m_);
            job_ = &f;
            parts_ = parts;
            next_.store(0);
            pending_ = (int)th_.size();
            ++gen_;
        }
        cv_.notify_all();
        for (int k; (k = next_.fetch_add(1)) < parts;) f(k);
        std::unique_lock<std::mutex> lk(m_);
        done_.wait(lk, [&] { return pending_ == 0; });
        job_ = nullptr;
    }

private:
    void loop()
    {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(m_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
            if (stop_) return;
            seen = gen_;
            const std::function<void(int)> *f = job_;
            const int parts = parts_;
            lk.unlock();
            for (int k; (k = next_.fetch_add(1)) < parts;) (*f)(k);
            lk.lock();
            if (--pending_ == 0) done_.notify_one();
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(int)> *job_ = nullptr;
    int parts_ = 0, pending_ = 0;
    std::atomic<int> next_{0};
    uint64_t gen_ = 0;
    bool stop_ = false;
};

struct Pending {
    uint64_t ticket;
    tersoff_request req;
    int64_t t_start;   // max(submit time, release time)
    CellGrid g;
    int ncell;
    bool pos_dev, types_dev, forces_dev;   // the request's buffers in this GPU's memory
};

// One configuration of a batch with a buffer in device memory: its device
// positions and / or types (null: staged from host memory) are copied into
// the batch by k_copy_inputs, its forces (null: returned through host
// staging) out of the batch by k_copy_outputs.
struct DevCopy {
    const double *pos;
    const int *types;
    double *forces;
    int off, n;
};

// Device-resident inputs into the batch arrays, one workgroup per
// configuration: positions and types copied as they are, a non-finite
// position (replaced by 0) or a type outside [0, ntypes) (replaced by 0)
// marks the configuration invalid in status[c] (written for every listed
// configuration), so no kernel of the batch ever indexes the parameter table
// with an unchecked type.
__global__ void k_copy_inputs(const DevCopy *__restrict__ list, int count, int ntypes, double *__restrict__ pos,
                              int *__restrict__ types, int *__restrict__ status)
{
    for (int c = blockIdx.x; c < count; c += gridDim.x) {
        const DevCopy d = list[c];
        int bad = 0;
        for (int a = threadIdx.x; a < d.n; a += blockDim.x) {
            const size_t o = (size_t)(d.off + a);
            if (d.pos) {
                double x = d.pos[3 * (size_t)a], y = d.pos[3 * (size_t)a + 1], z = d.pos[3 * (size_t)a + 2];
                if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
                    bad = 1;
                    x = y = z = 0.0;
                }
                pos[3 * o] = x;
                pos[3 * o + 1] = y;
                pos[3 * o + 2] = z;
            }
            if (d.types) {
                int t = d.types[a];
                if (t < 0 || t >= ntypes) {
                    bad = 1;
                    t = 0;
                }
                types[o] = t;
            }
        }
        bad = __syncthreads_or(bad);
        if (threadIdx.x == 0) status[c] = bad;
        __syncthreads();
    }
}

// Forces of the batch out to device-resident force arrays.
__global__ void k_copy_outputs(const DevCopy *__restrict__ list, int count, const double *__restrict__ forces)
{
    for (int c = blockIdx.x; c < count; c += gridDim.x) {
        const DevCopy d = list[c];
        if (!d.forces) continue;
        for (int k = threadIdx.x; k < 3 * d.n; k += blockDim.x) d.forces[k] = forces[3 * (size_t)d.off + k];
    }
}

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipGraphExec_t exec[kNumPrec] = {};   // one per precision
    Pinned<double> h_pos, h_forces, h_out;
    Pinned<int> h_types, h_sys_of;
    Pinned<SysDesc> h_desc;
    Pinned<BatchDims> h_dims;
    Pinned<DevCopy> h_copies;    // configurations of the batch with device-resident buffers
    Pinned<int> h_in_status;     // their input status (k_copy_inputs)
    Dev<DevCopy> copies;
    Dev<int> in_status;
    int ncopies = 0;
    bool dev_outputs = false;
    std::vector<int> copy_of;    // batch index -> copy list index (-1: none)
    Dev<double> pos, cell_pos, own, planes, forces, eatom, out;
    Dev<float4> cell_posf;
    Dev<int> long_rows;
    Dev<int> types, sys_of, cell_of, rank, cell_count, cell_start, cell_atoms, slot_cell, scan_tmp;
    Dev<int> ell, row_count, pcount, drop_list;   // ell: neighbour rows, row i at i * cap
    Dev<int> kept;   // kept-neighbour lists: A x kKeptFast, then A x kRecCap
    Dev<int> ctl;   // [0] flags, [1] dropped count, [2] long rows, [3 ..] per-system status
    Dev<unsigned char> recs;
    Dev<SysDesc> desc;
    Dev<BatchDims> dims;
    std::vector<Pending> batch;
    int natoms = 0;
    int prec = 0;
    bool want_forces = false;    // some configuration returns forces through host staging
    bool busy = false;
};

}  // namespace

struct Server {
    ServerEnv env{};
    int max_atoms = 0, max_sys = 0, max_cells = 0, cap = 0;
    double rc = 0.0;
    size_t max_queued = 0;
    size_t device_bytes = 0;
    int grids[kNumPrec][4] = {};
    Lane lanes[kLanes];
    std::unique_ptr<CopyPool> pool;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, tersoff_result> results;
    std::unordered_set<uint64_t> live;   // submitted, result not yet collected
    uint64_t next_ticket = 1;
    bool stopping = false;
    double n_batches = 0, n_systems = 0, n_atoms = 0;
};

namespace {

#define SRV_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return e_;               \
    } while (0)

// Cell grid of one box: cells at least rc wide (as in the single-system
// build), at most 1024 per axis.
CellGrid grid_of(const double box[3], double rc, long long &ncell)
{
    CellGrid g{};
    ncell = 1;
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
    return g;
}

hipError_t alloc_lane(Server &S, Lane &L)
{
    const size_t A = (size_t)S.max_atoms, NS = (size_t)S.max_sys, NC = (size_t)S.max_cells;
    const size_t E = A * (size_t)S.cap;
    size_t &tot = S.device_bytes;
    SRV_TRY(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
    SRV_TRY(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
    SRV_TRY(L.h_pos.alloc(3 * A));
    SRV_TRY(L.h_forces.alloc(3 * A));
    SRV_TRY(L.h_out.alloc(8 * NS));
    SRV_TRY(L.h_types.alloc(A));
    SRV_TRY(L.h_sys_of.alloc(A));
    SRV_TRY(L.h_desc.alloc(NS));
    SRV_TRY(L.h_dims.alloc(1));
    SRV_TRY(L.h_copies.alloc(NS));
    SRV_TRY(L.h_in_status.alloc(NS));
    SRV_TRY(L.pos.alloc(3 * A, tot));
    SRV_TRY(L.cell_pos.alloc(3 * A, tot));
    SRV_TRY(L.cell_posf.alloc(A + kPosPad, tot));
    SRV_TRY(L.long_rows.alloc(A, tot));
    SRV_TRY(L.own.alloc(3 * A, tot));
    SRV_TRY(L.planes.alloc(3 * (size_t)kRecCap * A, tot));
    SRV_TRY(L.forces.alloc(3 * A, tot));
    SRV_TRY(L.eatom.alloc(8 * A, tot));
    SRV_TRY(L.out.alloc(8 * NS, tot));
    SRV_TRY(L.types.alloc(A, tot));
    SRV_TRY(L.sys_of.alloc(A, tot));
    SRV_TRY(L.cell_of.alloc(A, tot));
    SRV_TRY(L.rank.alloc(A, tot));
    SRV_TRY(L.cell_count.alloc(NC, tot));
    SRV_TRY(L.cell_start.alloc(NC + 1, tot));
    SRV_TRY(L.cell_atoms.alloc(A, tot));
    SRV_TRY(L.slot_cell.alloc(A, tot));
    SRV_TRY(L.scan_tmp.alloc(std::max(scan_tmp_size((int)NC), scan_tmp_size((int)A)), tot));
    SRV_TRY(L.ell.alloc(E, tot));
    SRV_TRY(L.row_count.alloc(A, tot));
    SRV_TRY(L.kept.alloc((size_t)(kKeptFast + kRecCap) * A, tot));
    SRV_TRY(L.pcount.alloc(A, tot));
    SRV_TRY(L.drop_list.alloc(A, tot));
    SRV_TRY(L.ctl.alloc(3 + NS, tot));
    const size_t nbat = (A + kServeBatchAtoms - 1) / kServeBatchAtoms;
    const size_t slots = (size_t)kRecCap * nbat * kServeBatchAtoms;
    SRV_TRY(L.recs.alloc(std::max(record_region_bytes(kPrecFP64, slots), record_region_bytes(kPrecMixed, slots)),
                         tot));
    SRV_TRY(L.desc.alloc(NS, tot));
    SRV_TRY(L.copies.alloc(NS, tot));
    SRV_TRY(L.in_status.alloc(NS, tot));
    SRV_TRY(L.dims.alloc(1, tot));
    // every kept list starts empty (-1)
    SRV_TRY(hipMemsetAsync(L.kept.p, 0xff, sizeof(int) * (kKeptFast + kRecCap) * A, L.stream));
    SRV_TRY(hipMemsetAsync(L.pcount.p, 0, sizeof(int) * A, L.stream));
    return hipStreamSynchronize(L.stream);
}

void free_lane(Lane &L)
{
    for (auto &x : L.exec)
        if (x) (void)hipGraphExecDestroy(x), x = nullptr;
    L.h_pos.release(); L.h_forces.release(); L.h_out.release(); L.h_types.release();
    L.h_sys_of.release(); L.h_desc.release(); L.h_dims.release(); L.h_copies.release(); L.h_in_status.release();
    L.pos.release(); L.cell_pos.release(); L.own.release(); L.planes.release(); L.forces.release();
    L.cell_posf.release(); L.long_rows.release();
    L.eatom.release(); L.out.release(); L.types.release(); L.sys_of.release(); L.cell_of.release();
    L.rank.release(); L.cell_count.release(); L.cell_start.release(); L.cell_atoms.release();
    L.slot_cell.release();
    L.scan_tmp.release(); L.ell.release(); L.row_count.release(); L.kept.release();
    L.pcount.release();
    L.drop_list.release(); L.ctl.release(); L.recs.release(); L.desc.release(); L.copies.release();
    L.in_status.release();
    L.dims.release();
    if (L.done) (void)hipEventDestroy(L.done), L.done = nullptr;
    if (L.stream) (void)hipStreamDestroy(L.stream), L.stream = nullptr;
}

// The device work of one batch, enqueued on the lane's stream (captured once
// per precision; no allocation, no memset nodes, no host synchronisation).
hipError_t enqueue_batch(Server &S, Lane &L, int prec)
{
    hipStream_t s = L.stream;
    const int *n_dev = &L.dims.p->n_atoms;
    SRV_TRY(launch_fill_zero_int(L.cell_count.p, (size_t)S.max_cells, s));
    SRV_TRY(launch_fill_zero_int(L.ctl.p, 3 + (size_t)S.max_sys, s));
    SRV_TRY(launch_bin_systems(L.pos.p, L.sys_of.p, L.desc.p, L.dims.p, S.max_atoms, L.cell_of.p, L.rank.p,
                               L.cell_count.p, s));
    SRV_TRY(launch_exclusive_scan(L.cell_count.p, L.cell_start.p, S.max_cells, L.scan_tmp.p, nullptr, s));
    ScatterLaunch sca{};
    sca.pos = L.pos.p;
    sca.n = S.max_atoms;
    sca.cell_of = L.cell_of.p;
    sca.rank = L.rank.p;
    sca.cell_start = L.cell_start.p;
    sca.cell_atoms = L.cell_atoms.p;
    sca.slot_cell = L.slot_cell.p;
    sca.cell_pos = L.cell_pos.p;
    sca.cell_posf = L.cell_posf.p;
    sca.sys = L.desc.p;
    sca.sys_of = L.sys_of.p;
    sca.dims = L.dims.p;
    SRV_TRY(launch_scatter_cells(sca, kBatchGrid, s));
    SearchLaunch sl{};
    sl.sys = L.desc.p;
    sl.sys_of = L.sys_of.p;
    sl.dims = L.dims.p;
    sl.n = S.max_atoms;
    sl.rc2 = S.rc * S.rc;
    sl.rcs = (float)S.rc;
    sl.cell_start = L.cell_start.p;
    sl.cell_count = L.cell_count.p;
    sl.cell_atoms = L.cell_atoms.p;
    sl.slot_cell = L.slot_cell.p;
    sl.cell_of = L.cell_of.p;
    sl.cell_pos = L.cell_pos.p;
    sl.cell_posf = L.cell_posf.p;
    sl.cap = S.cap;
    sl.ell = L.ell.p;
    sl.row_count = L.row_count.p;
    sl.long_rows = L.long_rows.p;
    sl.n_long = L.ctl.p + 2;
    sl.sys_status = L.ctl.p + 3;
    SRV_TRY(launch_search(sl, kBatchGrid, s));

    PackLaunch pk{};
    pk.pos = L.pos.p;
    pk.types = L.types.p;
    pk.row_count = L.row_count.p;
    pk.ell = L.ell.p;
    pk.cap = S.cap;
    pk.n = S.max_atoms;
    pk.recs = L.recs.p;
    pk.rlo = rlo_of(L.recs.p, prec, (size_t)kRecCap * ((S.max_atoms + kServeBatchAtoms - 1) / kServeBatchAtoms) *
                                        kServeBatchAtoms);
    pk.pcount = L.pcount.p;
    pk.kept = L.kept.p;
    pk.kept_more = L.kept.p + (size_t)kKeptFast * S.max_atoms;
    pk.own = L.own.p;
    pk.flags = L.ctl.p;
    pk.drop_list = L.drop_list.p;
    pk.drop_count = L.ctl.p + 1;
    pk.pos_build = L.pos.p;
    pk.stale_sq = 0.0;
    pk.atoms_per_batch = kServeBatchAtoms;
    pk.n_dev = n_dev;
    pk.sys = L.desc.p;
    pk.sys_of = L.sys_of.p;
    SRV_TRY(launch_pack(pk, S.env.tab, prec, S.grids[prec][0], s));

    ComputeLaunch a{};
    a.types = L.types.p;
    a.recs = L.recs.p;
    a.rlo = pk.rlo;
    a.pcount = L.pcount.p;
    a.kept = L.kept.p;
    a.n = S.max_atoms;
    a.own = L.own.p;
    a.planes = L.planes.p;
    a.atoms_per_batch = kServeBatchAtoms;
    a.plane_stride = S.max_atoms;
    a.n_dev = n_dev;
    a.eatom = L.eatom.p;
    SRV_TRY(launch_compute(a, S.env.tab, prec, S.grids[prec][1], s));
    SRV_TRY(launch_fixup_dropped(L.ell.p, S.cap, L.row_count.p, L.kept.p, pk.kept_more, L.drop_list.p,
                                 L.ctl.p + 1, S.max_atoms, prec, L.planes.p, s));
    SRV_TRY(launch_gather_forces(L.pcount.p, prec, L.planes.p, L.own.p, S.max_atoms, n_dev, S.max_atoms, L.forces.p,
                                 nullptr, nullptr, FinalizeArgs{}, s));
    SRV_TRY(launch_reduce_systems(L.desc.p, L.dims.p, S.max_sys, L.eatom.p, L.drop_list.p, L.ctl.p + 1,
                                  L.ctl.p + 3, L.out.p, s));
    return hipSuccess;
}

hipError_t capture(Server &S, Lane &L, int prec)
{
    hipGraph_t g = nullptr;
    SRV_TRY(hipStreamBeginCapture(L.stream, hipStreamCaptureModeRelaxed));
    const hipError_t e = enqueue_batch(S, L, prec);
    const hipError_t e2 = hipStreamEndCapture(L.stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e != hipSuccess ? e : e2;
    }
    const hipError_t e3 = hipGraphInstantiate(&L.exec[prec], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e3;
}

// Takes requests from the head of the queue while they are released, share
// the head's precision and fit the atom, slot and cell capacities (called with
// the lock held).
void form_batch(Server &S, Lane &L)
{
    L.batch.clear();
    const int64_t now = now_ns();
    int natoms = 0, ncell = 0;
    while (!S.queue.empty() && (int)L.batch.size() < S.max_sys) {
        const Pending &p = S.queue.front();
        if (p.t_start > now) break;
        if (!L.batch.empty() && p.req.precision != L.prec) break;
        if (natoms + p.req.n > S.max_atoms || ncell + p.ncell > S.max_cells) break;
        if (L.batch.empty()) L.prec = p.req.precision;
        natoms += (int)p.req.n;
        ncell += p.ncell;
        L.batch.push_back(p);
        S.queue.pop_front();
    }
}

hipError_t launch_lane(Server &S, Lane &L)
{
    int off = 0, coff = 0;
    L.want_forces = false;
    L.dev_outputs = false;
    L.ncopies = 0;
    const int nsys = (int)L.batch.size();
    L.copy_of.assign(nsys, -1);
    for (int q = 0; q < nsys; ++q) {
        const Pending &p = L.batch[q];
        const int n = (int)p.req.n;
        SysDesc &d = L.h_desc.p[q];
        d.g = p.g;
        d.atom_off = off;
        d.natoms = n;
        d.cell_off = coff;
        d.pad = 0;
        if (p.pos_dev || p.types_dev || p.forces_dev) {
            DevCopy &c = L.h_copies.p[L.ncopies];
            c.pos = p.pos_dev ? p.req.pos : nullptr;
            c.types = p.types_dev ? p.req.types : nullptr;
            c.forces = p.forces_dev ? p.req.forces : nullptr;
            c.off = off;
            c.n = n;
            L.copy_of[q] = L.ncopies++;
            L.dev_outputs |= p.forces_dev;
        }
        off += n;
        coff += p.ncell;
        L.want_forces |= p.req.forces != nullptr && !p.forces_dev;
    }
    // host-resident inputs into pinned staging (device-resident ones are
    // copied on the device after the bulk upload, over the same range)
    S.pool->run(nsys, [&](int q) {
        const Pending &p = L.batch[q];
        const size_t n = (size_t)p.req.n, o = (size_t)L.h_desc.p[q].atom_off;
        if (!p.pos_dev) std::memcpy(L.h_pos.p + 3 * o, p.req.pos, sizeof(double) * 3 * n);
        if (!p.types_dev) std::memcpy(L.h_types.p + o, p.req.types, sizeof(int) * n);
        std::fill(L.h_sys_of.p + o, L.h_sys_of.p + o + n, q);
    });
    L.natoms = off;
    *L.h_dims.p = BatchDims{off, coff, nsys, 0};
    hipStream_t s = L.stream;
    SRV_TRY(hipMemcpyAsync(L.pos.p, L.h_pos.p, sizeof(double) * 3 * (size_t)off, hipMemcpyHostToDevice, s));
    SRV_TRY(hipMemcpyAsync(L.types.p, L.h_types.p, sizeof(int) * (size_t)off, hipMemcpyHostToDevice, s));
    SRV_TRY(hipMemcpyAsync(L.sys_of.p, L.h_sys_of.p, sizeof(int) * (size_t)off, hipMemcpyHostToDevice, s));
    SRV_TRY(hipMemcpyAsync(L.desc.p, L.h_desc.p, sizeof(SysDesc) * (size_t)nsys, hipMemcpyHostToDevice, s));
    SRV_TRY(hipMemcpyAsync(L.dims.p, L.h_dims.p, sizeof(BatchDims), hipMemcpyHostToDevice, s));
    if (L.ncopies) {
        SRV_TRY(hipMemcpyAsync(L.copies.p, L.h_copies.p, sizeof(DevCopy) * (size_t)L.ncopies, hipMemcpyHostToDevice,
                               s));
        hipLaunchKernelGGL(k_copy_inputs, dim3(std::min(L.ncopies, kBatchGrid)), dim3(256), 0, s, L.copies.p,
                           L.ncopies, S.env.ntypes, L.pos.p, L.types.p, L.in_status.p);
        SRV_TRY(hipGetLastError());
    }
    SRV_TRY(hipGraphLaunch(L.exec[L.prec], s));
    SRV_TRY(hipMemcpyAsync(L.h_out.p, L.out.p, sizeof(double) * 8 * (size_t)nsys, hipMemcpyDeviceToHost, s));
    if (L.ncopies)
        SRV_TRY(hipMemcpyAsync(L.h_in_status.p, L.in_status.p, sizeof(int) * (size_t)L.ncopies,
                               hipMemcpyDeviceToHost, s));
    if (L.want_forces)
        SRV_TRY(hipMemcpyAsync(L.h_forces.p, L.forces.p, sizeof(double) * 3 * (size_t)off, hipMemcpyDeviceToHost,
                               s));
    if (L.dev_outputs) {
        hipLaunchKernelGGL(k_copy_outputs, dim3(std::min(L.ncopies, kBatchGrid)), dim3(256), 0, s, L.copies.p,
                           L.ncopies, L.forces.p);
        SRV_TRY(hipGetLastError());
    }
    return hipEventRecord(L.done, s);
}

// Results of a finished (or failed) batch to the waiting callers.
void retire(Server &S, Lane &L, hipError_t status)
{
    const size_t nsys = L.batch.size();
    std::vector<std::pair<uint64_t, tersoff_result>> out(nsys);
    S.pool->run((int)nsys, [&](int q) {
        const Pending &p = L.batch[q];
        tersoff_result r{};
        r.tag = p.req.tag;
        r.n = p.req.n;
        r.batch_systems = (int32_t)nsys;
        if (status != hipSuccess) {
            r.status = TERSOFF_E_DEVICE;
        } else {
            const double *o = L.h_out.p + 8 * (size_t)q;
            const int st = (int)o[7];
            const int cq = L.copy_of[q];
            if (cq >= 0 && L.h_in_status.p[cq]) r.status = TERSOFF_E_INVALID;   // device input rejected
            else r.status = st ? TERSOFF_E_OVERFLOW : TERSOFF_OK;
            r.energy = o[0];
            for (int c = 0; c < 6; ++c) r.virial[c] = o[1 + c];
            if (p.req.forces && !p.forces_dev)
                std::memcpy(p.req.forces, L.h_forces.p + 3 * (size_t)L.h_desc.p[q].atom_off,
                            sizeof(double) * 3 * (size_t)p.req.n);
        }
        out[q] = {p.ticket, r};
    });
    // ready now: every force array of the batch has been written
    const int64_t now = now_ns();
    for (size_t q = 0; q < nsys; ++q) out[q].second.latency_ms = 1e-6 * (double)(now - L.batch[q].t_start);
    {
        std::lock_guard<std::mutex> lk(S.mu);
        for (auto &pr : out) S.results[pr.first] = pr.second;
        S.n_batches += 1;
        S.n_systems += (double)L.batch.size();
        S.n_atoms += (double)L.natoms;
    }
    S.cv_done.notify_all();
    L.batch.clear();
    L.busy = false;
}

void worker_main(Server *Sp)
{
    Server &S = *Sp;
    (void)hipSetDevice(S.env.device);
    std::deque<int> inflight;   // lanes in launch order
    for (;;) {
        while (!inflight.empty()) {
            Lane &L = S.lanes[inflight.front()];
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) break;
            retire(S, L, q);
            inflight.pop_front();
        }
        int free_lane = -1;
        for (int l = 0; l < kLanes; ++l)
            if (!S.lanes[l].busy) {
                free_lane = l;
                break;
            }
        if (free_lane >= 0) {
            Lane &L = S.lanes[free_lane];
            {
                std::unique_lock<std::mutex> lk(S.mu);
                form_batch(S, L);
                if (L.batch.empty() && inflight.empty()) {
                    if (S.stopping && S.queue.empty()) break;
                    if (S.queue.empty()) {
                        S.cv_work.wait(lk, [&] { return S.stopping || !S.queue.empty(); });
                    } else {
                        const int64_t wait = S.queue.front().t_start - now_ns();
                        if (wait > 0) S.cv_work.wait_for(lk, std::chrono::nanoseconds(wait));
                    }
                    continue;
                }
            }
            if (!L.batch.empty()) {
                L.busy = true;
                const hipError_t e = launch_lane(S, L);
                if (e != hipSuccess) {
                    (void)hipStreamSynchronize(L.stream);
                    retire(S, L, e);
                } else {
                    inflight.push_back(free_lane);
                }
                continue;
            }
        }
        if (inflight.empty()) continue;
        if (free_lane < 0) {
            (void)hipEventSynchronize(S.lanes[inflight.front()].done);
        } else {
            // a lane is free but nothing is ready: wake on a new request or
            // after a short interval to retire the running batch
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

}  // namespace

int server_create(const ServerEnv &env, const tersoff_serve_config &cfg, Server **out, std::string &err)
{
    *out = nullptr;
    const double cutoff = cfg.cutoff > 0 ? cfg.cutoff : env.max_cut;
    if (!(cutoff >= env.max_cut) || !(cfg.skin >= 0) || !std::isfinite(cfg.skin)) {
        err = "cutoff below the largest R + D, or negative skin";
        return TERSOFF_E_INVALID;
    }
    const int cap = cfg.max_neighbors > 0 ? ((cfg.max_neighbors + 7) / 8) * 8 : 48;
    if (cap > kMaxRow) {
        err = "max_neighbors above 256";
        return TERSOFF_E_INVALID;
    }
    if (cfg.max_batch_atoms < 1 || cfg.max_batch_atoms > (1 << 24) || cfg.max_batch_systems < 1 ||
        cfg.max_batch_systems > (1 << 20) || (long long)cfg.max_batch_atoms * cap >= (1LL << 31)) {
        err = "max_batch_atoms must be in [1, 2^24] with max_batch_atoms x row capacity < 2^31, "
              "max_batch_systems in [1, 2^20]";
        return TERSOFF_E_INVALID;
    }
    if (cfg.host_threads < 0 || cfg.host_threads > 64) {
        err = "host_threads must be in [0, 64]";
        return TERSOFF_E_INVALID;
    }
    Server *S = new (std::nothrow) Server();
    if (!S) return TERSOFF_E_NOMEM;
    S->env = env;
    S->max_atoms = (int)cfg.max_batch_atoms;
    S->max_sys = cfg.max_batch_systems;
    S->max_cells = std::max(S->max_atoms, 4096);
    S->cap = cap;
    S->rc = cutoff + cfg.skin;
    S->max_queued = cfg.max_queued > 0 ? (size_t)cfg.max_queued : 65536;
    for (int pr = 0; pr < kNumPrec; ++pr)
        compute_grids(pr, env.tab, true, S->max_atoms, kServeBatchAtoms, S->grids[pr]);
    hipError_t e = hipSetDevice(env.device);
    for (int l = 0; l < kLanes && e == hipSuccess; ++l) e = alloc_lane(*S, S->lanes[l]);
    for (int l = 0; l < kLanes && e == hipSuccess; ++l)
        for (int pr = 0; pr < kNumPrec && e == hipSuccess; ++pr) e = capture(*S, S->lanes[l], pr);
    if (e != hipSuccess) {
        err = std::string("serving set-up: ") + hipGetErrorString(e);
        for (auto &L : S->lanes) free_lane(L);
        delete S;
        return e == hipErrorOutOfMemory ? TERSOFF_E_NOMEM : TERSOFF_E_DEVICE;
    }
    try {
        S->pool.reset(new CopyPool(cfg.host_threads > 0 ? cfg.host_threads - 1 : 3));
        S->worker = std::thread(worker_main, S);
    } catch (...) {
        for (auto &L : S->lanes) free_lane(L);
        delete S;
        err = "cannot start the serving thread";
        return TERSOFF_E_DEVICE;
    }
    *out = S;
    return TERSOFF_OK;
}

void server_destroy(Server *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->env.device);
    for (auto &L : S->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        free_lane(L);
    }
    delete S;
}

// Where a buffer lives: 1 in the memory of `device`, 0 host memory (also
// memory the runtime does not know, and managed memory, which the host
// reads directly), -1 the memory of another GPU.
static int residency(const void *ptr, int device)
{
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
        (void)hipGetLastError();   // an unregistered host pointer
        return 0;
    }
    if (at.type != hipMemoryTypeDevice || at.isManaged) return 0;
    return at.device == device ? 1 : -1;
}

int server_submit(Server *S, const tersoff_request &req, uint64_t *ticket, std::string &err)
{
    if (!req.pos || !req.types || req.n < 1) {
        err = "request needs positions, types and n >= 1";
        return TERSOFF_E_INVALID;
    }
    if (req.n > S->max_atoms) {
        err = "request larger than the batch capacity";
        return TERSOFF_E_INVALID;
    }
    if (req.precision != TERSOFF_FP64 && req.precision != TERSOFF_MIXED && req.precision != TERSOFF_SINGLE) {
        err = "precision must be TERSOFF_FP64, TERSOFF_MIXED or TERSOFF_SINGLE";
        return TERSOFF_E_INVALID;
    }
    for (int a = 0; a < 3; ++a) {
        if (!(req.box[a] > 0) || !std::isfinite(req.box[a])) {
            err = "box must be positive";
            return TERSOFF_E_INVALID;
        }
        if (req.box[a] < 2.0 * S->rc) {
            err = "box length below 2 (cutoff + skin)";
            return TERSOFF_E_BOX;
        }
    }
    Pending p{};
    int res[3];
    const void *ptrs[3] = {req.pos, req.types, req.forces};
    for (int k = 0; k < 3; ++k) {
        res[k] = ptrs[k] ? residency(ptrs[k], S->env.device) : 0;
        if (res[k] < 0) {
            err = "a request buffer is device memory of another GPU";
            return TERSOFF_E_INVALID;
        }
    }
    p.pos_dev = res[0] == 1;
    p.types_dev = res[1] == 1;
    p.forces_dev = res[2] == 1;
    // host-resident inputs are checked here; device-resident ones by
    // k_copy_inputs (the result then reports E_INVALID)
    for (int64_t i = 0; i < req.n; ++i) {
        if (!p.types_dev && (req.types[i] < 0 || req.types[i] >= S->env.ntypes)) {
            err = "type out of range";
            return TERSOFF_E_INVALID;
        }
        if (!p.pos_dev && (!std::isfinite(req.pos[3 * i]) || !std::isfinite(req.pos[3 * i + 1]) ||
                           !std::isfinite(req.pos[3 * i + 2]))) {
            err = "non-finite position";
            return TERSOFF_E_INVALID;
        }
    }
    p.req = req;
    long long ncell = 0;
    p.g = grid_of(req.box, S->rc, ncell);
    if (ncell > S->max_cells) {
        err = "box has more cells than a batch holds";
        return TERSOFF_E_INVALID;
    }
    p.ncell = (int)ncell;
    const int64_t now = now_ns();
    p.t_start = std::max<int64_t>(now, req.release_ns);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping) {
            err = "server is stopping";
            return TERSOFF_E_STATE;
        }
        if (S->queue.size() >= S->max_queued) {
            err = "queue full";
            return TERSOFF_E_AGAIN;
        }
        p.ticket = S->next_ticket++;
        S->queue.push_back(p);
        S->live.insert(p.ticket);
    }
    S->cv_work.notify_one();
    *ticket = p.ticket;
    return TERSOFF_OK;
}

int server_poll(Server *S, uint64_t ticket, tersoff_result *res, double timeout_ms, std::string &err)
{
    std::unique_lock<std::mutex> lk(S->mu);
    if (!S->live.count(ticket)) {
        err = "unknown ticket (never issued, or its result was already collected)";
        return TERSOFF_E_INVALID;
    }
    auto ready = [&] { return S->results.count(ticket) != 0; };
    if (!ready() && timeout_ms > 0) {
        const auto until = std::chrono::steady_clock::now() +
                           std::chrono::nanoseconds((int64_t)(timeout_ms * 1e6));
        S->cv_done.wait_until(lk, until, ready);
    }
    auto it = S->results.find(ticket);
    if (it == S->results.end()) return TERSOFF_E_PENDING;
    *res = it->second;
    S->results.erase(it);
    S->live.erase(ticket);
    return TERSOFF_OK;
}

void server_stats(Server *S, double out[6])
{
    std::lock_guard<std::mutex> lk(S->mu);
    out[0] = S->n_batches;
    out[1] = S->n_systems;
    out[2] = S->n_atoms;
    out[3] = (double)S->device_bytes;
    out[4] = (double)S->max_atoms;
    out[5] = (double)S->max_sys;
}

}  // namespace tsf

extern "C" int64_t tersoff_clock_ns(void) { return tsf::now_ns(); }
