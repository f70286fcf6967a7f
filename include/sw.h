/*
 * swmi -- Swendsen-Wang multi-cluster sweep of the 2D q-state Potts model on one
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The operation (Komura & Okabe, "Multi-GPU-based Swendsen-Wang multi-cluster
 * algorithm for the simulation of two-dimensional q-state Potts model"):
 *   Sec. 2, Eq. (1): H = -J sum_<ij> (delta(S_i, S_j) - 1) on an L x L square
 *   lattice with periodic boundaries; one SW sweep = (1) activate bonds,
 *   (2) label the clusters of active bonds, (3) set every cluster to a random
 *   one of the q states.  The proper label of a cluster is its smallest label
 *   (Sec. 2, Hoshen-Kopelman paragraph), so cluster roots are minimum site
 *   indices.  Energy and magnetisation are measured after each sweep (Sec. 4,
 *   Table 1, "update + measurement").
 *
 * Fixed conventions (readings where the paper is silent):
 *   site index i = y*L + x; spins 0..q-1 (uint8); each site owns its bonds to
 *   (x+1, y) and (x, y+1) (periodic), 2N bonds in all; an equal-spin bond is
 *   active iff w < floor(2^32 (1 - e^{-K})), w a Philox4x32-10 draw keyed
 *   key = (seed lo, seed hi), bond counter (i >> 1, 0, sweep, 0) with words
 *   2(i&1) (+x) and 2(i&1)+1 (+y); the new state of a cluster with root r is
 *   floor(w q / 2^32), w = word 0 of counter (r, 0, sweep, 1); a random start
 *   uses word 0 of counter (i, 0, 0, 2) the same way.  Sweeps are numbered
 *   0, 1, 2, ... from sw_init.
 *
 * Memory and streams: the caller owns the device workspace (one allocation of
 * sw_workspace_bytes(), 256-byte aligned) and the HIP stream; both must stay
 * alive until sw_destroy.  The library never allocates device memory.  A handle
 * is bound to one stream and is not thread safe.  Host buffers are ordinary
 * (pageable) host memory owned by the caller.
 *
 * Errors: every int function returns SW_OK (0) or a negative SW_E* code and
 * never throws; sw_last_error() gives a message for the calling thread.
 * Work is asynchronous on the stream: sw_sweep returns before the GPU is done,
 * and a failure detected inside a kernel surfaces at the next call that
 * synchronises (sw_measure, sw_read_*).
 */
#ifndef SWMI_SW_H
#define SWMI_SW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SW_OK 0
#define SW_EINVAL (-1)     /* bad argument: L < 2 or > 65536, q < 2 or > 255, K < 0 or NaN, ... */
#define SW_ESPACE (-2)     /* workspace too small or not 256-byte aligned */
#define SW_EHIP (-3)       /* HIP runtime error; text in sw_last_error() */
#define SW_ESTATE (-4)     /* sweep counter would pass 2^32 - 1, or data not available */
#define SW_ECONVERGE (-5)  /* a labelling loop hit its safety cap (a bug detector) */

/* Parameters of one lattice. */
typedef struct sw_params {
    uint32_t L;            /* linear size, 2..65536 (N = L*L <= 2^32 sites) */
    uint32_t q;            /* number of Potts states, 2..255 */
    double K;              /* coupling J / k_B T, >= 0; +inf allowed (p = 1) */
    uint64_t seed;         /* Philox key */
    uint32_t init;         /* 0 = cold start (all spins 0), 1 = random start */
    uint32_t obs_capacity; /* sweeps of observables kept in the device ring;
                              0 = no measurement ("update only"), else >= 2 */
    uint32_t tile_rows;    /* labelling tile height: 32, 64 or 128; SW_TILE_WHOLE
                              (L <= 128, no cluster sums): the whole lattice in
                              one workgroup's LDS, many sweeps per launch; 0
                              (default): SW_TILE_WHOLE where it applies, else 64 */
    uint32_t flags;        /* 0, or SW_CLUSTER_SUMS */
} sw_params;

/* tile_rows: sweep the lattice whole in one workgroup's local memory (bonds,
 * union-find labels and new states of every sweep without a kernel launch per
 * sweep or global traffic between sweeps; the same random streams and cluster
 * keys as the tile kernels, so the same results).  Labels and bond words of a
 * call's last sweep are written for sw_read_labels / sw_read_bonds as usual. */
#define SW_TILE_WHOLE 1u

/* flags: also measure, for every sweep, the cluster-size sums of the sweep's
 * clusters (sw_cluster_sums).  Needs L <= 32768 and obs_capacity > 0. */
#define SW_CLUSTER_SUMS 1u

typedef struct sw_lattice sw_lattice;
typedef struct sw_batch sw_batch;
typedef struct sw_group sw_group;

/* Device bytes one lattice needs; 0 if the parameters are invalid. */
size_t sw_workspace_bytes(const sw_params* p);

/* Integer bond threshold floor(2^32 (1 - e^{-K})) in [0, 2^32] (bond
 * probability of Sec. 2 step (1) as an integer test on a 32-bit draw). */
int sw_threshold(const sw_params* p, uint64_t* thr);

/* State of Sec. 2: the spins S_i of Eq. (1) (here 0..q-1) on the L x L torus.
 * The paper does not say how a run starts; init = 0 sets every spin to 0,
 * init = 1 draws each spin from its own counter (see the keying above).
 * Carves the lattice out of dev_ws (device pointer, ws_bytes bytes, 256-byte
 * aligned: SW_ESPACE otherwise) and writes the initial spins on hip_stream (a
 * hipStream_t; NULL = default stream), then synchronises.  *out receives a
 * host-side handle owned by the library (freed by sw_destroy).  Bad
 * parameters: SW_EINVAL, and *out is NULL. */
int sw_init(const sw_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, sw_lattice** out);

/* Enqueue n_sweeps SW sweeps (Sec. 2 steps (1)-(3)) on the handle's stream,
 * each followed by the measurement of energy and state counts when
 * obs_capacity > 0.  Asynchronous. */
int sw_sweep(sw_lattice* h, uint32_t n_sweeps);

/* Observables of sweeps first .. first+n-1 (after each sweep's flip), copied
 * into host_out as n rows of (2 + q) int64: [n_unsat, n_active, n_0, ...,
 * n_{q-1}], where n_unsat = number of unsatisfied bonds (energy of Eq. (1) in
 * units of J), n_active = bonds activated in that sweep, n_c = sites in state
 * c.  Only the last obs_capacity sweeps since sw_init / sw_load_spins are
 * kept.  Synchronises the stream. */
int sw_measure(sw_lattice* h, uint32_t first, uint32_t n, int64_t* host_out);

/* Cluster-size sums of sweeps first .. first+n-1 (lattices made with
 * SW_CLUSTER_SUMS), for the improved estimators of the moments of the
 * magnetisation behind the moment ratio of Sec. 4: given a sweep's clusters C,
 * the mean over their independent uniform new states of |M|^2 (M the simplex-
 * vector magnetisation, the Ising M for q = 2) is S2 = sum_C |C|^2, and that
 * of |M|^4 is (1 + 2/(q-1)) S2^2 - (2/(q-1)) S4 with S4 = sum_C |C|^4.
 * host_out: n rows of 3 uint64: S2, then S4 as 128 bits (low word, high
 * word).  Same availability rules as sw_measure (SW_ESTATE also without the
 * flag).  Synchronises the stream. */
int sw_cluster_sums(sw_lattice* h, uint32_t first, uint32_t n, uint64_t* host_out);

/* sw_sweep with timing: HIP events are recorded on the handle's stream around
 * every kernel launch; the call then synchronises and writes the summed device
 * time of each phase, in milliseconds, into phase_ms[5]: [0] bonds + tile
 * labels (+ measurement of the incoming configuration), [1] tile-edge merge,
 * [2] flip, [3] final measurement and counter update, [4] the part of [0]
 * spent in the model's bond kernel (the XY model's k_xy_bonds; for the Potts
 * model, whose bonds and labels are one kernel, equal to [0]).  The results
 * are the same as sw_sweep's. */
int sw_sweep_profiled(sw_lattice* h, uint32_t n_sweeps, double* phase_ms);

/* sw_measure and sw_read_spins on a stream other than the handle's, for a
 * caller that keeps the handle's stream busy with further sweeps meanwhile
 * (continuous batching: the results of one step are read while the next runs;
 * no paper counterpart).  read_stream (a hipStream_t, not NULL) first waits for
 * after_event (a hipEvent_t recorded on the handle's stream after the sweeps
 * to be read, or NULL), then sums the ring records / copies the spins and
 * synchronises read_stream only.  The caller must not let later sweeps pass
 * the records being read (obs_capacity) or touch the spins being read.
 * Same arguments and errors as sw_measure / sw_read_spins otherwise. */
int sw_measure_after(sw_lattice* h, void* read_stream, void* after_event, uint32_t first, uint32_t n,
                     int64_t* host_out);
int sw_read_spins_after(sw_lattice* h, void* read_stream, void* after_event, uint8_t* host_out);

/* Number of sweeps done since sw_init (the index of the next sweep). */
int sw_sweeps_done(const sw_lattice* h, uint32_t* out);

/* The spins S_i of Eq. (1) after the last sweep (states 0..q-1), N bytes
 * row-major (i = y*L + x) into caller-owned host memory.  Synchronises the
 * stream; a kernel that tripped a safety cap gives SW_ECONVERGE. */
int sw_read_spins(sw_lattice* h, uint8_t* host_out);

/* Checkpoint / resume of the Markov chain of Sec. 2: replace the spins with
 * host_in (N bytes row-major, each < q: SW_EINVAL otherwise, nothing changed)
 * and set the sweep counter to `sweep`, so that the next sweep draws exactly
 * what sweep number `sweep` of an uninterrupted run draws.  Observables before
 * `sweep` are dropped.  Synchronises the stream. */
int sw_load_spins(sw_lattice* h, const uint8_t* host_in, uint32_t sweep);

/* Cluster labels of the last sweep (the labelling of Sec. 2 step (2), each
 * cluster labelled by its smallest site index as in the Hoshen-Kopelman
 * paragraph): N uint32, label[i] = smallest site index of i's cluster.  Needs
 * at least one sweep since init / load.  Synchronises. */
int sw_read_labels(sw_lattice* h, uint32_t* host_out);

/* The bonds activated in step (1) of the last sweep (Sec. 2) as two bit planes
 * (+x, then +y), each L rows of ceil(L/64) uint64 words; bit (x mod 64) of
 * word x/64 of row y is the bond of site (x, y); padding bits are 0.
 * 2 * L * ceil(L/64) words of caller-owned host memory.  Needs a sweep since
 * init / load (SW_ESTATE otherwise).  Synchronises. */
int sw_read_bonds(sw_lattice* h, uint64_t* host_out);

/* Comparison only (no sweep uses it): the labelling scheme the paper builds
 * on, iterated label equivalence (Sec. 2, the scan and analysis kernels
 * repeated under a host loop until a scan changes no label), run on the
 * active bonds of the last sweep.  dev_labels: caller-owned device buffer of
 * N uint32 that receives label[i] = smallest site index of i's cluster (the
 * same labels sw_read_labels gives); dev_flag: one caller-owned device uint32
 * (scratch).  *iterations receives the number of scan + analysis passes,
 * counting the last one, which changed nothing; *ms (if not NULL) the
 * elapsed device time of the whole loop, host round trips included.  More
 * than max_iter passes: SW_ECONVERGE.  Needs a sweep since init / load;
 * synchronises the stream; leaves the lattice unchanged. */
int sw_label_equivalence(sw_lattice* h, uint32_t* dev_labels, uint32_t* dev_flag, uint32_t max_iter,
                         uint32_t* iterations, double* ms);

/* Release the handle (not the workspace or the stream). */
int sw_destroy(sw_lattice* h);

/* ---------------------------------------------------------------- batched
 * Many independent lattices ("replicas") of uneven L, q and K swept by the
 * same kernels in one launch per phase.  The paper sweeps one lattice at a
 * time; a batch runs that same sweep (Sec. 2 steps (1)-(3)) on every replica.
 * Replica r behaves bit for bit like a plain lattice with params[r] (same
 * random draws: nothing but the replica's own seed and sweep index keys them).
 * Same conventions as the plain calls: caller-owned workspace and stream,
 * asynchronous sweeps, synchronising reads, negative SW_E* codes. */

/* Device bytes for the n replicas params[0..n-1] (each checked as by
 * sw_workspace_bytes; all must have the same tile_rows: SW_EINVAL). */
int sw_batch_workspace_bytes(const sw_params* params, uint32_t n, size_t* bytes);

/* As sw_init for every replica, in one workspace of sw_batch_workspace_bytes()
 * bytes (256-byte aligned).  Synchronises the stream. */
int sw_batch_init(const sw_params* params, uint32_t n, void* dev_ws, size_t ws_bytes,
                  void* hip_stream, sw_batch** out);

/* Sweep replica r n_sweeps[r] times (0 = leave it alone); n_sweeps is n host
 * uint32.  Asynchronous. */
int sw_batch_sweep(sw_batch* b, const uint32_t* n_sweeps);

/* Same sweep count for every replica, captured once per count as a HIP graph
 * and replayed (a few counts are cached per batch; the count is a constant of
 * its graph).  On the legacy NULL stream, which cannot be captured, the kernels
 * are launched directly.  Asynchronous. */
int sw_batch_sweep_all(sw_batch* b, uint32_t n_sweeps);

/* sw_measure, sw_read_spins, sw_cluster_sums, sw_sweeps_done and sw_destroy
 * for one replica (replica >= n: SW_EINVAL). */
int sw_batch_measure(sw_batch* b, uint32_t replica, uint32_t first, uint32_t n, int64_t* host_out);
int sw_batch_read_spins(sw_batch* b, uint32_t replica, uint8_t* host_out);
int sw_batch_cluster_sums(sw_batch* b, uint32_t replica, uint32_t first, uint32_t n, uint64_t* host_out);
int sw_batch_sweeps_done(const sw_batch* b, uint32_t replica, uint32_t* out);
int sw_batch_destroy(sw_batch* b);

/* Tile-height autotuner.  The labelling tile height (tile_rows) only splits the
 * connected-component labelling of Sec. 2 step (2) between the tile-local pass
 * and the tile-edge merge (the two stages of Sec. 3); spins, labels and
 * observables do not depend on it (cluster roots are smallest site indices and
 * every draw is keyed by site and sweep), so it is a pure performance choice.
 * For each of the n_candidates (1..8) heights in candidates[] (each 32, 64,
 * 128, SW_TILE_WHOLE -- every replica swept whole in LDS, which needs
 * L <= 128 and no cluster sums -- or 0, the default rule: whole where that
 * applies, 64 elsewhere), this initialises the n replicas params[] (their own
 * tile_rows is ignored) in dev_ws, runs `sweeps` (1..4096) untimed sweeps of every replica,
 * then times `sweeps` more with HIP events on hip_stream, and writes the
 * fastest height into *tile_rows and, if ms_per_sweep is not NULL, the measured
 * milliseconds per sweep of candidate c into ms_per_sweep[c].  dev_ws must hold
 * sw_batch_workspace_bytes() of the replicas at every candidate height (checked
 * before any launch: SW_ESPACE); its contents are overwritten and no handle
 * survives the call.  Synchronises the stream. */
int sw_batch_autotune(const sw_params* params, uint32_t n, const uint32_t* candidates, uint32_t n_candidates,
                      uint32_t sweeps, void* dev_ws, size_t ws_bytes, void* hip_stream, uint32_t* tile_rows,
                      double* ms_per_sweep);

/* ----------------------------------------------------------------- groups
 * Continuous batching: one launch per phase over any set of lattices made by
 * sw_init (same tile_rows, same stream), which may change from call to call.
 * Each lattice is swept exactly as sw_sweep would (same random draws). */

/* Tiles of one lattice (the unit of work of every launch). */
int sw_tile_count(const sw_params* p, uint32_t* tiles);

/* Device bytes of a group's scratch for up to max_lattices lattices holding up
 * to max_tiles tiles in total. */
int sw_group_workspace_bytes(uint32_t max_lattices, uint64_t max_tiles, size_t* bytes);

/* A group (no paper counterpart: the sweep of Sec. 2 on many resident
 * lattices at once) with its scratch in dev_ws (sw_group_workspace_bytes()
 * bytes, 256-byte aligned, caller-owned) on hip_stream.  tile_rows: 0
 * (default), 32, 64 or 128; members must match it. */
int sw_group_init(uint32_t max_lattices, uint64_t max_tiles, uint32_t tile_rows, void* dev_ws, size_t ws_bytes,
                  void* hip_stream, sw_group** out);

/* Sweep lats[i] n_sweeps[i] times (0 = leave it alone), i < n, every lattice
 * at most once, bound to the group's stream; each is swept exactly as
 * sw_sweep would (Sec. 2 steps (1)-(3)).  Asynchronous. */
int sw_group_sweep(sw_group* g, sw_lattice* const* lats, const uint32_t* n_sweeps, uint32_t n);

/* Release the group's handle (not its workspace, stream or lattices). */
int sw_group_destroy(sw_group* g);

/* Energy and order parameter of Sec. 4 ("energy and magnetization", measured
 * after each sweep) in FP64 from one observable row of sw_measure for an
 * L x L lattice with q states: out[0] = n_unsat / N (energy per site of
 * Eq. (1) in units of J), out[1] = (q max_c n_c / N - 1) / (q - 1) (Potts
 * order parameter), out[2] = n_0 - n_1 for q = 2 (Ising magnetisation; 0 for
 * other q).  row: 2 + q host int64; out: 3 host doubles.  Bad L or q, or a row
 * whose counts do not add up to N: SW_EINVAL. */
int sw_derived(uint32_t L, uint32_t q, const int64_t* row, double* out);

/* ------------------------------------------------- no-allocation variant
 * For callers that cannot allocate device memory or set up a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  sw_sweep + sw_measure in one call that uses no workspace: the
 * labels, bond words, edge records, observable ring, sweep counter and
 * descriptor live in one fixed array of SW_STATIC_SCRATCH_BYTES of device
 * memory that the library holds on every GPU it runs on until the process
 * ends.  It calls no hipMalloc / hipFree and no allocating library routine,
 * and enqueues only kernel launches, so it can be captured in a graph.
 *
 * p: L, q, K, seed, tile_rows as for sw_init (init and obs_capacity are
 * checked as there but not used).  dev_spins: device, N bytes row-major,
 * states < q (not checked), read and overwritten in place.  first_sweep:
 * index of the first sweep (keys its draws exactly as sweep number
 * first_sweep of a lattice made by sw_init).  dev_obs: device, n_sweeps rows
 * of (2 + q) int64 as sw_measure gives them, or NULL for no measurement.
 * dev_status: device uint32 that receives 0, or nonzero if a labelling safety
 * cap tripped, or NULL.  Asynchronous on hip_stream; results are bit-identical
 * to sw_init + sw_load_spins(spins, first_sweep) + sw_sweep + sw_measure.
 * Errors: SW_EINVAL (parameters), SW_ESTATE (first_sweep + n_sweeps > 2^32-1),
 * SW_ESPACE if the lattice needs more than SW_STATIC_SCRATCH_BYTES (about
 * 4.3 bytes per site: L <= 2048 always fits), SW_EHIP.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (other streams, other threads) race and give wrong results.  Each call
 * clears what must start at zero (ring, counter, error flag) itself. */
#define SW_STATIC_SCRATCH_BYTES (24u << 20)
int sw_sweep_static(const sw_params* p, uint8_t* dev_spins, uint32_t first_sweep, uint32_t n_sweeps,
                    int64_t* dev_obs, uint32_t* dev_status, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* sw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SWMI_SW_H */
