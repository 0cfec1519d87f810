/*
 * tersoff.h -- C ABI of libtersoff.so: Tersoff many-body energy, forces and
 * virial on one AMD Instinct MI355X (gfx950).
 *
 * The method is the Tersoff potential as restated in Section 2 of Hoehnerbach,
 * Ismail and Bientinesi, "The Tersoff many-body potential: sustainable
 * performance through vectorization":
 *   Eq. (1)  E = 1/2 sum_i sum_{j: r_ij < R+D} f_C(r_ij) [f_R(r_ij) + b_ij f_A(r_ij)]
 *   Eq. (2)  b_ij = (1 + beta^eta zeta_ij^eta)^(-1/(2 eta))
 *   Eq. (3)  zeta_ij = sum_{k != j: r_ik < R+D} f_C(r_ik) g(theta_ijk) exp((lambda3 (r_ij - r_ik))^m)
 * with f_C(r) = 1 below R-D, 1/2 - 1/2 sin(pi/2 (r-R)/D) up to R+D, 0 beyond;
 * f_R = A exp(-lambda1 r); f_A = -B exp(-lambda2 r);
 * g = gamma (1 + c^2/d^2 - c^2/(d^2 + (cos theta - h)^2)).
 * Forces follow Algorithm 1: zeta_ij over k, then V(i,j,zeta_ij) and its
 * derivative on i and j, then dV/dzeta * d zeta(i,j,k)/dx on i, j and k.
 * The neighbour list with a skin and the packing of in-cutoff entries are the
 * scheme of Sections 2 and 3.
 *
 * Units: eV and Angstrom.  F = -dE/dx.  Virial W_ab = sum over all pair and
 * triplet force terms of r_a F_b with r the relative vector from the centre
 * atom (eV; positive = repulsive); reported as xx yy zz xy xz yz.
 *
 * Every call returns a tersoff_status (0 = OK, negative = error); no call
 * aborts or throws across this boundary.  A context is used by one host
 * thread at a time; the serving calls (tersoff_submit / tersoff_poll) are
 * thread-safe.
 */
#ifndef TERSOFF_H
#define TERSOFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One parameter-table entry is 14 doubles in this order. */
#define TERSOFF_NPARAM 14
enum {
    TERSOFF_P_A = 0,       /* eV                          */
    TERSOFF_P_B = 1,       /* eV                          */
    TERSOFF_P_LAMBDA1 = 2, /* 1/A                         */
    TERSOFF_P_LAMBDA2 = 3, /* 1/A                         */
    TERSOFF_P_LAMBDA3 = 4, /* 1/A                         */
    TERSOFF_P_BETA = 5,
    TERSOFF_P_ETA = 6,     /* Tersoff's n                 */
    TERSOFF_P_C = 7,
    TERSOFF_P_D = 8,
    TERSOFF_P_H = 9,       /* cos(theta_0)                */
    TERSOFF_P_GAMMA = 10,
    TERSOFF_P_R = 11,      /* A, centre of the switch     */
    TERSOFF_P_DC = 12,     /* A, half-width of the switch */
    TERSOFF_P_M = 13       /* 1 or 3 (exponent of Eq. 3)  */
};
#define TERSOFF_MAX_TYPES 4

/* TERSOFF_FP64: all FP64.  TERSOFF_MIXED: FP32 pair and triplet functions;
 * FP64 displacement, zeta -> b_ij power in log form, and every accumulation
 * of energy, force and virial.  TERSOFF_SINGLE: as mixed, but the zeta -> b_ij
 * power and each pair's sum of force terms in FP32 too (FP64 only for the
 * displacement and the sums across pairs and atoms); the paper's "single"
 * point (Section 5). */
typedef enum { TERSOFF_FP64 = 0, TERSOFF_MIXED = 1, TERSOFF_SINGLE = 2 } tersoff_precision;

typedef enum {
    TERSOFF_OK = 0,
    TERSOFF_E_INVALID = -1,  /* bad argument or parameter                    */
    TERSOFF_E_NOMEM = -2,    /* device allocation failed                     */
    TERSOFF_E_BOX = -3,      /* a box length is below 2 (cutoff + skin)      */
    TERSOFF_E_OVERFLOW = -4, /* an atom has more in-range neighbours than
                                the kernel's per-batch capacity              */
    TERSOFF_E_STALE = -5,    /* an atom moved more than skin/2 since build   */
    TERSOFF_E_DEVICE = -6,   /* HIP runtime error                            */
    TERSOFF_E_AGAIN = -7,    /* serving: no slot or memory free right now    */
    TERSOFF_E_PENDING = -8,  /* serving: result not ready yet                */
    TERSOFF_E_STATE = -9     /* call out of order (e.g. compute before build)*/
} tersoff_status;

typedef struct tersoff_ctx tersoff_ctx;

/* Create a context on the current HIP device.
 * params: host array of ntypes^3 entries (entry (ti,tj,tk) at
 *   ((ti*ntypes + tj)*ntypes + tk) * TERSOFF_NPARAM), copied.  Pair terms and
 *   (beta, eta) of a bond i-j use entry (t_i, t_j, t_j); the zeta term of k and
 *   the cutoff applied to r_ik use entry (t_i, t_j, t_k).
 * Errors: E_INVALID if ntypes is not in [1, TERSOFF_MAX_TYPES], or an entry
 *   has A <= 0, B <= 0, D <= 0, R - D < 0, eta <= 0, beta < 0, c or d == 0,
 *   m not 1 or 3, or a non-finite value;
 *   E_NOMEM / E_DEVICE. */
int tersoff_create(const double *params, int32_t ntypes, tersoff_ctx **out);

/* Release every device buffer of the context.  NULL is ignored. */
void tersoff_destroy(tersoff_ctx *ctx);

/* Full neighbour list (Section 2: every j != i with minimum-image
 * r_ij < cutoff + skin, skin atoms included), built on the GPU with a cell
 * list; rows sorted by j.  The minimum-image displacement is, per axis,
 * s = rint(d/L), d' = fma(-s, L, d), and r^2 = fma(dz,dz, fma(dy,dy, dx*dx)).
 * pos: device, n x 3 float64 (row-major); types: device, n int32 in
 *   [0, ntypes); positions need not be wrapped into the box.
 * box: host, 3 orthorhombic periodic lengths.  cutoff must be >= the largest
 *   R + D of the table; skin >= 0.
 * stream: hipStream_t or NULL.  The call synchronises that stream (it reads
 *   back the list length).  pos and types are copied; the list and the copies
 *   stay resident in the context until the next build.  When fewer than half
 *   of the consecutive atoms of the caller's order lie in the same or
 *   adjacent cells, the context also keeps the list in the cell order's
 *   numbering, and tersoff_compute works in that numbering (positions
 *   permuted in, forces written back at the caller's indices): results do
 *   not depend on the caller's order beyond floating-point summation order.
 * Errors: E_INVALID (n < 1 or > 2^24, cutoff too small, type out of range,
 *   non-finite position), E_BOX (a box length < 2 (cutoff + skin)),
 *   E_OVERFLOW (an atom has more than 256 neighbours within cutoff + skin),
 *   E_NOMEM, E_DEVICE.  Rows longer than the working capacity are handled by
 *   a retry with a larger capacity. */
int tersoff_build_neighbors(tersoff_ctx *ctx, const double *pos, const int32_t *types,
                            int64_t n, const double box[3], double cutoff, double skin,
                            void *stream);

/* Energy, forces and virial (Eq. 1-3, Algorithm 1) from the resident list.
 * pos: device, n x 3 float64 for the same n atoms as the last build (they may
 *   have moved; the minimum-image displacement is recomputed in FP64).
 * precision: TERSOFF_FP64, TERSOFF_MIXED or TERSOFF_SINGLE (tersoff_precision).
 * energy_virial: device, 7 float64 written: E, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz.
 * forces: device, n x 3 float64, overwritten; may be NULL.
 * Stream-ordered on `stream`; does not synchronise.  A capacity overflow or a
 * stale list detected on the device is reported by tersoff_check.
 * Errors (host-side): E_STATE (no list), E_INVALID (precision), E_DEVICE. */
int tersoff_compute(tersoff_ctx *ctx, const double *pos, int32_t precision,
                    double *energy_virial, double *forces, void *stream);

/* tersoff_compute without allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The same evaluation as tersoff_compute
 * (the same kernels in the same launch configuration: results identical bit
 * for bit), with every per-evaluation buffer -- records, force planes,
 * per-atom forces and counts, kept-neighbour lists, partial sums, the
 * positions in the internal numbering (see tersoff_build_neighbors), and the
 * force output when forces is NULL -- taken from one fixed device array of
 * the library (about 34 MB on each GPU it runs on, held from the first use of
 * the library's device code on that GPU until the process ends) instead of
 * the context.  The call allocates nothing; the neighbour list comes from
 * tersoff_build_neighbors (which does allocate), for at most
 * TERSOFF_STATIC_MAX_ATOMS atoms.  Every call on one GPU shares the array
 * (whatever its context or stream): calls that overlap on one GPU race.
 * Arguments, ownership and errors as tersoff_compute, plus E_INVALID when the
 * last build has more than TERSOFF_STATIC_MAX_ATOMS atoms. */
#define TERSOFF_STATIC_MAX_ATOMS 16384
int tersoff_compute_static(tersoff_ctx *ctx, const double *pos, int32_t precision,
                           double *energy_virial, double *forces, void *stream);

/* Synchronise `stream` and report the device-side status of every compute
 * since the previous check: OK, E_OVERFLOW (an atom exceeded the per-batch
 * neighbour capacity; its terms were skipped), E_STALE (an atom moved more
 * than skin/2 from its position at the last build) or E_DEVICE (a centre
 * kept a neighbour that did not keep it back -- an internal invariant, not
 * an input condition).  Clears the flags. */
int tersoff_check(tersoff_ctx *ctx, void *stream);

/* Copy the resident neighbour list to host memory (synchronises).
 * offsets: host, n+1 int64; idx: host, cap int32; *total receives the list
 * length.  If cap < total only offsets and *total are written and
 * E_INVALID is returned. */
int tersoff_get_neighbors(tersoff_ctx *ctx, int64_t *offsets, int32_t *idx, int64_t cap,
                          int64_t *total);

/* Work counts of the last compute (synchronises): counts[0] = list entries S,
 * counts[1] = in-cutoff ordered pairs P, counts[2] = ordered triplets T
 * (centre i, j and k in cutoff, k != j). */
int tersoff_get_counts(tersoff_ctx *ctx, int64_t counts[3]);

/* Kernel timing with HIP events on the caller's stream.  While enabled, every
 * tersoff_compute records event pairs around its packing kernel, its main
 * (energy / force / virial) kernel, and its per-atom plus force-gather
 * kernels, and every tersoff_build_neighbors one pair around its whole device
 * work.  tersoff_profile_read synchronises the device and returns, then
 * resets, summed times (ms) and counts: out[0] main kernel, out[1] its
 * launches, out[2] builds, out[3] their number, out[4] per-atom + gather,
 * out[5] their launches, out[6] packing, out[7] its launches. */
int tersoff_profile(tersoff_ctx *ctx, int32_t enable);
int tersoff_profile_read(tersoff_ctx *ctx, double out[8]);

/* Nominal centre atoms per wavefront batch of the compute kernel, in
 * [1, 64] (default: chosen by each build, 32, or 16 below 131,072 atoms;
 * once set, kept for later builds).  Performance tuning only; results do not
 * depend on it beyond floating-point summation order.  E_INVALID outside
 * the range. */
int tersoff_set_batch_atoms(tersoff_ctx *ctx, int32_t atoms);

/* How tersoff_compute sums the force terms (Section 3: the pair-vectorised
 * scheme makes lanes of one vector update the same atoms).  mode 0 (the
 * default): every term of centre i on atom j is summed by the lane of pair
 * (i, j) and stored in a force plane of j, then each atom adds its planes in
 * a fixed order -- no atomics, results reproducible bit for bit.  mode 1: the
 * same terms added with FP64 atomics into the zeroed force array (no planes,
 * no gather; the summation order, hence the last bits, vary from run to run)
 * -- the comparison point of mode 0.  Both agree within the stated
 * tolerances.  E_INVALID for another mode. */
int tersoff_set_force_sum(tersoff_ctx *ctx, int32_t mode);

/* Where tersoff_compute packs each centre's neighbours (the kept entries of
 * its row with their FP64 minimum-image displacements, Section 2's full list
 * with a skin).  mode 0 (the default): a separate packing kernel writes the
 * packed records, each atom's kept-neighbour list and its count, which the
 * compute kernel reads.  mode 1: the compute kernel packs each group of
 * centre atoms itself, into a queue in LDS, and stores each force term in
 * the plane of the centre's position in the neighbour's row (no records,
 * kept lists or counts pass through memory) -- a comparison point, slower
 * on the measured workloads; it applies when every row of the last build
 * holds at most 64 entries, with tersoff_set_mapping mode 0 and
 * tersoff_set_force_sum mode 0 (otherwise mode 0 runs).  Both give the same
 * forces bit for bit, energy and virial up to the order of their sums.
 * E_INVALID for another mode. */
int tersoff_set_packing(tersoff_ctx *ctx, int32_t mode);

/* How tersoff_compute maps the triplet loop onto the 64 lanes of a
 * wavefront (Section 3 compares vectorising over centre atoms with
 * vectorising over their neighbours; Table 2).  mode 0 (the default): a lane
 * per packed pair (i, j), with the pairs of several centre atoms side by side
 * in one batch; the lane runs the K loops of its pair.  mode 1: the same
 * batches with the lanes taken by the triplets (i; j, k) of the batch, zeta
 * and the force terms summed with LDS atomics (the order of those sums, hence
 * the last bits, vary from run to run) -- a comparison point, for
 * TERSOFF_FP64 and TERSOFF_MIXED with the force planes (tersoff_set_force_sum
 * mode 0).  A lane per neighbour of one centre atom is mode 0 with
 * tersoff_set_batch_atoms(ctx, 1).  E_INVALID for another mode; a later
 * tersoff_compute with TERSOFF_SINGLE or the atomic scatter under mode 1
 * returns E_INVALID. */
int tersoff_set_mapping(tersoff_ctx *ctx, int32_t mode);

/* Number of atoms of the last build (0 if none). */
int64_t tersoff_num_atoms(const tersoff_ctx *ctx);

/* Static text for a status code. */
const char *tersoff_strerror(int status);

/* Message of the last error raised on this context ("" if none). */
const char *tersoff_last_error(const tersoff_ctx *ctx);

/* ---- Serving: many small, independent configurations ------------------
 *
 * The evaluation of one configuration is Eq. (1)-(3) / Algorithm 1 on its
 * own periodic box, exactly as tersoff_build_neighbors + tersoff_compute
 * define it.  A worker thread of the context gathers queued requests into
 * batches (first come first served, up to the capacities below, one
 * precision per batch), builds every configuration's neighbour list and
 * evaluates the whole batch with one replay of a captured HIP graph, while
 * the next batch is formed from requests that arrived in the meantime.  A
 * configuration's result does not depend on which other configurations share
 * its batch.  A request's buffers may be host memory or device memory of the
 * context's GPU (told apart with hipPointerGetAttributes): host inputs are
 * staged through pinned memory, device inputs copied into the batch on the
 * device, forces written back to either.  The device memory of two batches
 * in flight is allocated once, at start, from the capacities. */
typedef struct {
    int64_t max_batch_atoms;    /* atoms per batch, in [1, 2^24]; also the largest request  */
    int32_t max_batch_systems;  /* configurations per batch (slots), in [1, 2^20]           */
    int32_t max_neighbors;      /* row capacity of a batch's lists (0: 48; at most 256); a
                                   configuration with a longer row gets E_OVERFLOW          */
    double cutoff;              /* 0: the largest R + D of the table                        */
    double skin;                /* list radius = cutoff + skin                              */
    int64_t max_queued;         /* waiting requests before submit returns E_AGAIN (0: 65536) */
    int32_t host_threads;       /* host threads copying requests in and results out,
                                   the worker included (0: 4)                               */
    int32_t reserved;           /* 0                                                        */
} tersoff_serve_config;

typedef struct {
    const double *pos;      /* host or device, n x 3 float64; read when the request
                               joins a batch                                             */
    const int32_t *types;   /* host or device, n int32 in [0, ntypes)                    */
    int64_t n;
    double box[3];          /* orthorhombic periodic lengths, each >= 2 (cutoff + skin)  */
    int32_t precision;      /* a tersoff_precision                                       */
    double *forces;         /* host or device, n x 3, written before the result is
                               ready; or NULL                                            */
    uint64_t tag;           /* returned unchanged                                        */
    int64_t release_ns;     /* tersoff_clock_ns() time before which the request is not
                               started (0: at once); latency counts from the later of
                               submission and release                                    */
} tersoff_request;

typedef struct {
    int32_t status;         /* OK, or E_OVERFLOW (a row above max_neighbors or an atom
                               above the per-atom record capacity: values invalid),
                               E_INVALID (device-resident input with a type out of range
                               or a non-finite position), or E_DEVICE                    */
    int32_t batch_systems;  /* configurations in the batch that evaluated it             */
    int64_t n;
    double energy;          /* eV                                                        */
    double virial[6];       /* xx yy zz xy xz yz, eV                                     */
    double latency_ms;      /* from submission (or release) to result ready              */
    uint64_t tag;
} tersoff_result;

/* Start the serving worker of a context (device memory for two batches is
 * allocated here).  Errors: E_INVALID (capacities, cutoff below the largest
 * R + D, skin < 0), E_STATE (already started), E_NOMEM, E_DEVICE. */
int tersoff_serve_start(tersoff_ctx *ctx, const tersoff_serve_config *cfg);

/* Finish every queued and running request, then stop the worker and free its
 * memory (tersoff_destroy does this too).  Results not yet collected are
 * dropped.  Errors: E_STATE (not started). */
int tersoff_serve_stop(tersoff_ctx *ctx);

/* Queue one configuration.  pos, types and forces must stay valid until its
 * result has been collected.  Thread-safe.
 * Errors: E_INVALID (null pointer, n < 1 or above max_batch_atoms, type out
 *   of range or non-finite position in host memory, non-finite box,
 *   precision, a box with more cells than a batch holds, a buffer in the
 *   memory of another GPU), E_BOX (a box length < 2 (cutoff + skin)),
 *   E_AGAIN (max_queued requests waiting), E_STATE (serving not started or
 *   stopping).  Device-resident inputs are checked on the device: a bad one
 *   yields a result with status E_INVALID. */
int tersoff_submit(tersoff_ctx *ctx, const tersoff_request *req, uint64_t *ticket);

/* Collect the result of a ticket, waiting up to timeout_ms (0: do not wait).
 * Returns OK (result written; the ticket is then retired), E_PENDING (not
 * ready yet), E_INVALID (unknown or already collected ticket) or E_STATE.
 * Thread-safe. */
int tersoff_poll(tersoff_ctx *ctx, uint64_t ticket, double timeout_ms, tersoff_result *res);

/* Serving counters: out[0] batches run, out[1] configurations, out[2] atoms,
 * out[3] device bytes held, out[4] max_batch_atoms, out[5] max_batch_systems. */
int tersoff_serve_stats(tersoff_ctx *ctx, double out[6]);

/* Monotonic clock (ns) of tersoff_request.release_ns. */
int64_t tersoff_clock_ns(void);

/* ---- Parameter files and a molecular-dynamics driver -------------------- */

/* Parse a parameter file in the LAMMPS "tersoff" format (the public format:
 * after '#' comments, a stream of 17-word entries -- elements i j k, then
 * m, gamma, lambda3, c, d, cos(theta0), n, beta, lambda2, B, R, D, lambda1,
 * A -- in any line layout; R and D as in Eq. (1), cutoff R + D).
 * elements: host, nelem names; type t is elements[t].  Entries naming other
 * elements are skipped.
 * params_out: host, nelem^3 * TERSOFF_NPARAM doubles in the layout of
 *   tersoff_create.
 * Errors: E_INVALID (null pointer, nelem outside [1, TERSOFF_MAX_TYPES], a
 *   word count that is not a multiple of 17, a malformed number, a triplet
 *   given twice or missing).  Host only; needs no device. */
int tersoff_parse_params(const char *text, const char *const *elements, int32_t nelem, double *params_out);

typedef struct {
    double dt;              /* time step, ps                                       */
    int32_t nsteps;         /* velocity-Verlet steps (>= 0)                        */
    int32_t precision;      /* a tersoff_precision                                 */
    const double *mass;     /* host, ntypes masses, amu                            */
    double cutoff;          /* 0: the largest R + D of the table                   */
    double skin;            /* > 0, A                                              */
} tersoff_md_config;

/* Constant-energy molecular dynamics around the evaluation: nsteps steps of
 * velocity Verlet in metal units (eV, A, ps, amu; acceleration
 * F / m * 9648.53321 A/ps^2 per eV/(A amu)).  The neighbour list is built at
 * the start and rebuilt before any step at which an atom has moved more than
 * skin/2 since the last build (the condition under which Section 2's skin
 * keeps the list complete).
 * pos, vel, forces: device, n x 3 float64, advanced in place; forces holds
 *   the forces of the final positions.  types: device, n int32.
 * out: host, 4 doubles: potential energy and kinetic energy (eV) of the final
 *   state, neighbour builds (the first included), temperature (K, 3N degrees
 *   of freedom).
 * The stream is synchronised once per step (the displacement check).
 * Errors: E_INVALID (arguments, masses <= 0, dt <= 0, skin <= 0), and those
 *   of tersoff_build_neighbors / tersoff_compute / tersoff_check. */
int tersoff_md_run(tersoff_ctx *ctx, double *pos, double *vel, double *forces, const int32_t *types, int64_t n,
                   const double box[3], const tersoff_md_config *cfg, double out[4], void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TERSOFF_H */
