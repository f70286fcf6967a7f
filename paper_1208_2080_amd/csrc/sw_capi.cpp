// C ABI of the SW sweep library: handle management, workspace carving, the
// fixed per-sweep kernel schedule and error mapping.  The library never
// allocates device memory; every device byte comes from the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sw.h"
#include "../../include/sw_xy.h"
#include "sw_kernels.hpp"
#include "sw_layout.hpp"

using namespace swmi;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(SW_EHIP, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

constexpr uint32_t DEFAULT_TY = 64;

// Validate parameters; on success fill the derived geometry.
struct Geometry {
    uint32_t L, q, W, ty, ntx, nty, ntiles, cap;
    size_t N;
    uint64_t thr;
    bool csum;   // cluster-size sums measured
    bool xy = false;         // an XY lattice (q unused)
    bool whole = false;      // swept whole in one workgroup's LDS (k_whole); ty is the bond-word layout
    uint32_t dir_bits = 0;   // XY: bits of the direction draw kept
    double K = 0.0;          // XY: the coupling
};

// Words of a ring record and of one partial copy's stride, for either model.
inline uint32_t rec_words(const Geometry& g) { return g.xy ? XY_WORDS : ring_words(g.q); }
inline uint32_t rec_stride(const Geometry& g) { return g.xy ? XY_STRIDE : ring_stride(g.q); }

uint64_t threshold_of(double K)
{
    if (std::isinf(K)) return 1ull << 32;
    const double p = -std::expm1(-K);    // bond probability 1 - e^{-K}
    return (uint64_t)std::floor(std::ldexp(p, 32));
}

// The geometry shared by both models: L, tile height, ring capacity.
int check_common(uint32_t L, uint32_t obs_capacity, uint32_t tile_rows, Geometry* g)
{
    if (L < 2 || L > 65536) return fail(SW_EINVAL, "L = %u outside 2..65536", L);
    if (obs_capacity == 1) return fail(SW_EINVAL, "obs_capacity must be 0 or >= 2");
    if (obs_capacity > (1u << 28)) return fail(SW_EINVAL, "obs_capacity too large");
    const uint32_t ty = (tile_rows == 0 || tile_rows == SW_TILE_WHOLE) ? DEFAULT_TY : tile_rows;
    if (ty != 32 && ty != 64 && ty != 128)
        return fail(SW_EINVAL, "tile_rows must be 0, SW_TILE_WHOLE, 32, 64 or 128");
    g->L = L;
    g->W = (L + 63) / 64;
    g->ty = ty;
    g->ntx = (L + TX - 1) / TX;
    g->nty = (L + ty - 1) / ty;
    g->ntiles = g->ntx * g->nty;
    g->cap = obs_capacity;
    g->N = (size_t)L * L;
    return SW_OK;
}

int check_xy_params(const sw_xy_params* p, Geometry* g)
{
    if (!p) return fail(SW_EINVAL, "params is NULL");
    if (std::isnan(p->K) || p->K < 0) return fail(SW_EINVAL, "K must be >= 0 (got %g)", p->K);
    if (p->dir_bits < 1 || p->dir_bits > 32) return fail(SW_EINVAL, "dir_bits = %u outside 1..32", p->dir_bits);
    if (p->init > 1) return fail(SW_EINVAL, "init must be 0 (cold) or 1 (random)");
    if (p->reserved) return fail(SW_EINVAL, "reserved must be 0");
    if (p->tile_rows == SW_TILE_WHOLE) return fail(SW_EINVAL, "SW_TILE_WHOLE sweeps Potts lattices only");
    const int rc = check_common(p->L, p->obs_capacity, p->tile_rows, g);
    if (rc) return rc;
    g->q = 0;
    g->thr = 0;
    g->csum = false;
    g->xy = true;
    g->dir_bits = p->dir_bits;
    g->K = p->K;
    return SW_OK;
}

int check_params(const sw_params* p, Geometry* g)
{
    if (!p) return fail(SW_EINVAL, "params is NULL");
    if (p->L < 2 || p->L > 65536) return fail(SW_EINVAL, "L = %u outside 2..65536", p->L);
    if (p->q < 2 || p->q > 255) return fail(SW_EINVAL, "q = %u outside 2..255", p->q);
    if (std::isnan(p->K) || p->K < 0) return fail(SW_EINVAL, "K must be >= 0 (got %g)", p->K);
    if (p->init > 1) return fail(SW_EINVAL, "init must be 0 (cold) or 1 (random)");
    const int rc = check_common(p->L, p->obs_capacity, p->tile_rows, g);
    if (rc) return rc;
    if (p->flags & ~SW_CLUSTER_SUMS) return fail(SW_EINVAL, "unknown flags 0x%x", p->flags);
    if ((p->flags & SW_CLUSTER_SUMS) && (p->L > 32768 || p->obs_capacity == 0))
        return fail(SW_EINVAL, "cluster sums need L <= 32768 and obs_capacity > 0");
    g->q = p->q;
    g->thr = threshold_of(p->K);
    g->csum = (p->flags & SW_CLUSTER_SUMS) != 0;
    const bool fits = p->L <= WHOLE_LMAX && !g->csum;
    if (p->tile_rows == SW_TILE_WHOLE && !fits)
        return fail(SW_EINVAL, "SW_TILE_WHOLE needs L <= %u and no cluster sums", WHOLE_LMAX);
    g->whole = p->tile_rows == SW_TILE_WHOLE || (p->tile_rows == 0 && fits);
    return SW_OK;
}

// The ring keeps one slot more than the sweeps it reports: the slot of the
// next sweep is cleared ahead of time by the flip kernel.
inline uint32_t ring_slots(const Geometry& g) { return g.cap ? g.cap + 1 : 0; }

// Byte offsets of one lattice's arrays inside its slice of the workspace.
struct Carve {
    size_t state, desc, spins, lab, bonds, edges, nodes, csize, ring, obs, total;
};

Carve carve(const Geometry& g)
{
    Carve c{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    c.state = take(sizeof(DevState));
    c.desc = take(sizeof(LatDesc));
    c.spins = take(g.xy ? g.N * 4 : g.N);
    c.lab = take(g.N * 4);
    c.bonds = take((size_t)g.ntiles * 2 * g.ty * 8);
    c.edges = take((size_t)g.ntiles * edge_words(g.ty) * 4);
    c.nodes = take((size_t)g.ntiles * nslot(g.ty) * 8);
    c.csize = take(g.csum ? (size_t)g.ntiles * nslot(g.ty) * 8 : 0);
    c.ring = take((size_t)ring_slots(g) * NCOPY * rec_stride(g) * 8);
    c.obs = take((size_t)ring_slots(g) * rec_words(g) * 8);
    c.total = off;
    return c;
}

// Multiply-high division by L (Granlund & Montgomery): l = ceil(log2 L).
void division_magic(uint32_t L, uint32_t* magic, uint32_t* shift)
{
    uint32_t l = 0;
    while ((1ull << l) < L) ++l;
    *magic = (uint32_t)((((1ull << l) - L) << 32) / L + 1);
    *shift = l - 1;
}

bool division_ok(uint32_t L, uint32_t magic, uint32_t shift)
{
    const uint32_t probes[] = {0u, 1u, L - 1, L, L + 1, 2 * L - 1, 0x7FFFFFFFu, 0x80000000u,
                               0xFFFFFFFEu, 0xFFFFFFFFu, (uint32_t)((uint64_t)L * L - 1), 123456789u};
    for (uint32_t n : probes) {
        const uint32_t t = (uint32_t)(((uint64_t)magic * n) >> 32);
        if (((t + ((n - t) >> 1)) >> shift) != n / L) return false;
    }
    return true;
}

LatDesc make_desc(const Geometry& g, uint64_t seed, char* base, const Carve& c)
{
    LatDesc d{};
    DevState* st = reinterpret_cast<DevState*>(base + c.state);
    if (g.xy) {
        d.ang = reinterpret_cast<uint32_t*>(base + c.spins);
        d.k2 = 2.0 * g.K;
        d.dir_keep = g.dir_bits >= 32 ? 0xFFFFFFFFu : ~(0xFFFFFFFFu >> g.dir_bits);
        d.xy = 1;
    } else {
        d.s = reinterpret_cast<uint8_t*>(base + c.spins);
    }
    d.lab = reinterpret_cast<uint32_t*>(base + c.lab);
    d.tlab = reinterpret_cast<uint16_t*>(base + c.lab + (size_t)g.N * 2);
    d.bonds = reinterpret_cast<uint64_t*>(base + c.bonds);
    d.edges = reinterpret_cast<uint32_t*>(base + c.edges);
    d.nodes = reinterpret_cast<uint64_t*>(base + c.nodes);
    d.csize = g.csum ? reinterpret_cast<uint64_t*>(base + c.csize) : nullptr;
    d.ring = g.cap ? reinterpret_cast<int64_t*>(base + c.ring) : nullptr;
    d.obs = g.cap ? reinterpret_cast<int64_t*>(base + c.obs) : nullptr;
    d.counter = &st->counter;
    d.err = &st->err;
    d.L = g.L;
    d.q = g.q;
    d.W = g.W;
    d.ntx = g.ntx;
    d.nty = g.nty;
    d.ntiles = g.ntiles;
    d.cap = ring_slots(g);
    d.thr_nz = g.thr != 0;
    d.thr_m1 = g.thr ? (uint32_t)(g.thr - 1) : 0u;
    d.key0 = (uint32_t)seed;
    d.key1 = (uint32_t)(seed >> 32);
    division_magic(g.L, &d.magic, &d.shift);
    d.log2L = 0;
    if ((g.L & (g.L - 1)) == 0)
        while ((1u << d.log2L) < g.L) ++d.log2L;
    return d;
}

// Captured sweeps: the first sweep of a call (nothing to measure before it),
// and the next ones one and STEP_CHUNK at a time.  Any number of sweeps
// replays these three graphs; kernels only, no copies or fills.
constexpr uint32_t STEP_CHUNK = 16;

struct StepGraphs {
    hipGraphExec_t first = nullptr, next = nullptr, chunk = nullptr;
    void clear()
    {
        for (hipGraphExec_t* g : {&first, &next, &chunk})
            if (*g) {
                (void)hipGraphExecDestroy(*g);
                *g = nullptr;
            }
    }
};

}  // namespace

// One lattice: host-side view of its slice of the workspace.
struct sw_lattice {
    Geometry g;
    Carve c;
    char* base;
    LatDesc desc;            // host copy of the descriptor
    LatDesc* d_desc;         // device copy (read by every kernel)
    hipStream_t stream;
    uint32_t done;           // sweeps done since init (index of the next sweep)
    uint32_t first_obs;      // first sweep whose observables exist
    bool have_sweep;         // labels and bonds of a sweep are in place
    bool labels_resolved;    // the label region holds all N smallest site indices (a whole-lattice sweep)
    StepGraphs graphs;       // captured sweeps (streams other than the legacy NULL stream)
};

namespace {

int check_device_error(const LatDesc& d, hipStream_t s)
{
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, d.err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err) return fail(SW_ECONVERGE, "a labelling loop hit its safety cap");
    return SW_OK;
}

// Rows of (2 + q) int64 for ring records [first, first+n): n_unsat, n_active,
// n_0..n_{q-1}.  A small kernel sums each record's NCOPY partial copies into
// the lattice's staging area, so only (q + 1) words per sweep cross to the
// host, in one copy and one synchronisation; n_0 = N - the other counts.
// With cs_out (n rows of 3 uint64): the cluster-size sums of the records,
// sum |C|^2 and the low and high words of sum |C|^4, instead of the rows.
int read_ring(const LatDesc& d, size_t N, hipStream_t s, uint32_t first, uint32_t n, int64_t* out,
              uint64_t* cs_out = nullptr)
{
    if (n == 0) return SW_OK;
    if (n >= d.cap) return fail(SW_ESTATE, "internal: %u records exceed the ring", n);
    const uint32_t W = d.xy ? XY_WORDS : ring_words(d.q);
    std::vector<int64_t> buf((size_t)n * W);
    HIP_TRY(launch_ring_sum(d.ring, d.obs, d.cap, first % d.cap, n, W, d.xy ? XY_STRIDE : ring_stride(d.q), s));
    HIP_TRY(hipMemcpyAsync(buf.data(), d.obs, buf.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (d.xy) {   // XY rows are the records themselves
        std::memcpy(out, buf.data(), buf.size() * 8);
        return SW_OK;
    }
    if (cs_out) {
        for (uint32_t k = 0; k < n; ++k)
            for (uint32_t j = 0; j < 3; ++j) cs_out[(size_t)k * 3 + j] = (uint64_t)buf[(size_t)k * W + cs_word(d.q) + j];
        return SW_OK;
    }
    for (uint32_t k = 0; k < n; ++k) {
        const int64_t* r = buf.data() + (size_t)k * W;
        int64_t* row = out + (size_t)k * (2 + d.q);
        row[0] = r[0];
        row[1] = r[1];
        int64_t rest = 0;
        for (uint32_t c = 1; c < d.q; ++c) {
            row[2 + c] = r[1 + c];
            rest += r[1 + c];
        }
        row[2] = (int64_t)N - rest;
    }
    return SW_OK;
}

// The phases of a sweep for either model: the bonds with the labelling
// (XY: the model's bond kernel, then the labeller over its bond words), the
// flip (XY: reflections), and the measurement of the last sweep's result.
int phase_bonds(const Work& w, uint32_t k, uint32_t flags, hipEvent_t after_bonds = nullptr)
{
    if (w.xy) {
        HIP_TRY(launch_xy_bonds(w, k, flags));
        if (after_bonds) HIP_TRY(hipEventRecord(after_bonds, w.stream));
        HIP_TRY(launch_label_preset(w));
    } else {
        HIP_TRY(launch_bond_label(w, k, flags));
        if (after_bonds) HIP_TRY(hipEventRecord(after_bonds, w.stream));
    }
    return SW_OK;
}

int phase_flip(const Work& w, uint32_t k)
{
    HIP_TRY(w.xy ? launch_flip_xy(w, k) : launch_flip(w, k));
    return SW_OK;
}

int phase_measure(const Work& w, uint32_t k)
{
    HIP_TRY(w.xy ? launch_xy_bonds(w, k, 2u) : launch_measure(w, k));
    return SW_OK;
}

// The fixed schedule of n sweeps on one Work description.  With ev (4n + 2
// events) an event is recorded before the first launch, after the bond kernel
// and after every phase.
int enqueue_sweeps(const Work& w, uint32_t n, bool measure, const LatDesc* descs, uint32_t count,
                   const uint32_t* n_each, hipEvent_t* ev = nullptr)
{
    if (ev) HIP_TRY(hipEventRecord(ev[0], w.stream));
    for (uint32_t k = 0; k < n; ++k) {
        int rc = phase_bonds(w, k, (measure && k > 0) ? 1u : 0u, ev ? ev[4 * k + 1] : nullptr);
        if (rc) return rc;
        if (ev) HIP_TRY(hipEventRecord(ev[4 * k + 2], w.stream));
        HIP_TRY(launch_merge(w));
        if (ev) HIP_TRY(hipEventRecord(ev[4 * k + 3], w.stream));
        rc = phase_flip(w, k);
        if (rc) return rc;
        if (w.cluster) HIP_TRY(launch_cluster_sums(w, k));
        if (ev) HIP_TRY(hipEventRecord(ev[4 * k + 4], w.stream));
    }
    if (measure) {
        const int rc = phase_measure(w, n - 1);
        if (rc) return rc;
    }
    HIP_TRY(launch_bump(descs, count, n_each, n, w.stream));
    if (ev) HIP_TRY(hipEventRecord(ev[4 * n + 1], w.stream));
    return SW_OK;
}

// One sweep of every lattice in w with its sweep counter bumped at the end,
// so that a captured step replays as the next sweep each time.  flags as for
// launch_bond_label (bit 0: measure the configuration the bonds are drawn on).
int enqueue_step(const Work& w, uint32_t flags, const LatDesc* descs, uint32_t count)
{
    int rc = phase_bonds(w, 0, flags);
    if (rc) return rc;
    HIP_TRY(launch_merge(w));
    rc = phase_flip(w, 0);
    if (rc) return rc;
    if (w.cluster) HIP_TRY(launch_cluster_sums(w, 0));
    HIP_TRY(launch_bump(descs, count, nullptr, 1, w.stream));
    return SW_OK;
}

int capture_steps(const Work& w, uint32_t flags, uint32_t steps, const LatDesc* descs, uint32_t count,
                  hipGraphExec_t* out)
{
    hipGraph_t graph;
    HIP_TRY(hipStreamBeginCapture(w.stream, hipStreamCaptureModeThreadLocal));
    int rc = SW_OK;
    for (uint32_t k = 0; k < steps && rc == SW_OK; ++k) rc = enqueue_step(w, flags, descs, count);
    const hipError_t ec = hipStreamEndCapture(w.stream, &graph);
    if (rc != SW_OK) return rc;
    if (ec != hipSuccess) return fail(SW_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(SW_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    return SW_OK;
}

// n sweeps from the captured steps (built on first use), then the
// measurement of the last sweep (the one before the bumped counter).
int run_steps(StepGraphs& G, const Work& w, uint32_t n, bool measure, const LatDesc* descs, uint32_t count)
{
    if (!G.first) {
        int rc = capture_steps(w, 0u, 1, descs, count, &G.first);
        if (rc == SW_OK) rc = capture_steps(w, measure ? 1u : 0u, 1, descs, count, &G.next);
        if (rc == SW_OK) rc = capture_steps(w, measure ? 1u : 0u, STEP_CHUNK, descs, count, &G.chunk);
        if (rc) {
            G.clear();
            return rc;
        }
    }
    HIP_TRY(hipGraphLaunch(G.first, w.stream));
    uint32_t left = n - 1;
    for (; left >= STEP_CHUNK; left -= STEP_CHUNK) HIP_TRY(hipGraphLaunch(G.chunk, w.stream));
    for (; left; --left) HIP_TRY(hipGraphLaunch(G.next, w.stream));
    if (measure) return phase_measure(w, 0xFFFFFFFFu);   // counter - 1: the last sweep
    return SW_OK;
}

}  // namespace

extern "C" {

const char* sw_last_error(void) { return g_err.c_str(); }

size_t sw_workspace_bytes(const sw_params* p)
{
    Geometry g;
    if (check_params(p, &g) != SW_OK) return 0;
    return carve(g).total;
}

int sw_threshold(const sw_params* p, uint64_t* thr)
{
    if (!p || !thr) return fail(SW_EINVAL, "NULL argument");
    if (std::isnan(p->K) || p->K < 0) return fail(SW_EINVAL, "K must be >= 0 (got %g)", p->K);
    *thr = threshold_of(p->K);
    return SW_OK;
}

// A lattice of either model in the caller's workspace: descriptor, cleared
// state and ring, initial spins (angles).
static int create_lattice(const Geometry& g, uint64_t seed, uint32_t random_start, void* dev_ws, size_t ws_bytes,
                          void* hip_stream, sw_lattice** out)
{
    const Carve c = carve(g);
    if (!dev_ws || ((uintptr_t)dev_ws % ALIGN) != 0)
        return fail(SW_ESPACE, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < c.total) return fail(SW_ESPACE, "workspace has %zu bytes, needs %zu", ws_bytes, c.total);
    sw_lattice* h = new (std::nothrow) sw_lattice();
    if (!h) return fail(SW_EINVAL, "out of host memory");
    h->g = g;
    h->c = c;
    h->base = static_cast<char*>(dev_ws);
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->desc = make_desc(g, seed, h->base, c);
    if (!division_ok(g.L, h->desc.magic, h->desc.shift)) {
        delete h;
        return fail(SW_EINVAL, "internal: division by L self-check failed");
    }
    h->d_desc = reinterpret_cast<LatDesc*>(h->base + c.desc);
    auto run = [&]() -> int {
        HIP_TRY(hipMemsetAsync(h->base + c.state, 0, sizeof(DevState), h->stream));
        HIP_TRY(hipMemcpyAsync(h->d_desc, &h->desc, sizeof(LatDesc), hipMemcpyHostToDevice, h->stream));
        if (g.cap) HIP_TRY(hipMemsetAsync(h->base + c.ring, 0, (size_t)ring_slots(g) * NCOPY * rec_stride(g) * 8, h->stream));
        if (g.csum) HIP_TRY(hipMemsetAsync(h->base + c.csize, 0, (size_t)g.ntiles * nslot(g.ty) * 8, h->stream));
        if (g.xy) HIP_TRY(launch_xy_init(h->d_desc, g.N, random_start, h->stream));
        else if (random_start) HIP_TRY(launch_init(h->d_desc, 0, g.N, 1u, h->stream));
        else HIP_TRY(hipMemsetAsync(h->desc.s, 0, g.N, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        return SW_OK;
    };
    const int rc = run();
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return SW_OK;
}

int sw_init(const sw_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, sw_lattice** out)
{
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    Geometry g;
    const int rc = check_params(p, &g);
    if (rc) return rc;
    return create_lattice(g, p->seed, p->init, dev_ws, ws_bytes, hip_stream, out);
}

// n sweeps of a lattice swept whole, in launches of at most WHOLE_CHUNK
// sweeps; the last sweep's labels and bond words are written.
constexpr uint32_t WHOLE_CHUNK = 4096;

static int whole_sweeps(sw_lattice* h, uint32_t n)
{
    for (uint32_t done = 0; done < n;) {
        const uint32_t k = std::min(WHOLE_CHUNK, n - done);
        HIP_TRY(launch_whole(h->d_desc, nullptr, 1, h->g.L, 0, k, nullptr, 1u, h->g.ty, h->stream));
        done += k;
    }
    h->done += n;
    h->have_sweep = true;
    h->labels_resolved = true;   // k_whole writes smallest site indices
    return SW_OK;
}

int sw_sweep(sw_lattice* h, uint32_t n_sweeps)
{
    if (!h) return fail(SW_EINVAL, "handle is NULL");
    if (n_sweeps == 0) return SW_OK;
    if ((uint64_t)h->done + n_sweeps > 0xFFFFFFFFull) return fail(SW_ESTATE, "sweep counter would overflow");
    if (h->g.whole) return whole_sweeps(h, n_sweeps);
    const Work w{h->d_desc, nullptr, h->g.ntiles, h->g.ty, h->stream, h->g.csum, h->g.xy};
    // the legacy NULL stream cannot be captured: launch directly
    const int rc = h->stream ? run_steps(h->graphs, w, n_sweeps, h->g.cap != 0, h->d_desc, 1)
                             : enqueue_sweeps(w, n_sweeps, h->g.cap != 0, h->d_desc, 1, nullptr);
    if (rc) return rc;
    h->done += n_sweeps;
    h->have_sweep = true;
    h->labels_resolved = false;
    return SW_OK;
}

int sw_sweep_profiled(sw_lattice* h, uint32_t n_sweeps, double* phase_ms)
{
    if (!h || !phase_ms) return fail(SW_EINVAL, "NULL argument");
    for (int i = 0; i < 5; ++i) phase_ms[i] = 0.0;
    if (n_sweeps == 0) return SW_OK;
    if ((uint64_t)h->done + n_sweeps > 0xFFFFFFFFull) return fail(SW_ESTATE, "sweep counter would overflow");
    if (n_sweeps > (1u << 20)) return fail(SW_EINVAL, "profile at most 2^20 sweeps per call");
    if (h->g.whole) {
        // one kernel does every phase: its time is the bond-and-label phase
        hipEvent_t e[2] = {nullptr, nullptr};
        for (auto& x : e) HIP_TRY(hipEventCreate(&x));
        int rc = SW_OK;
        if (hipEventRecord(e[0], h->stream) != hipSuccess) rc = fail(SW_EHIP, "hipEventRecord failed");
        if (rc == SW_OK) rc = whole_sweeps(h, n_sweeps);
        if (rc == SW_OK && hipEventRecord(e[1], h->stream) != hipSuccess) rc = fail(SW_EHIP, "hipEventRecord failed");
        if (rc == SW_OK && hipEventSynchronize(e[1]) != hipSuccess) rc = fail(SW_EHIP, "hipEventSynchronize failed");
        float ms = 0.f;
        if (rc == SW_OK && hipEventElapsedTime(&ms, e[0], e[1]) != hipSuccess)
            rc = fail(SW_EHIP, "hipEventElapsedTime failed");
        for (auto& x : e) (void)hipEventDestroy(x);
        if (rc) return rc;
        phase_ms[0] = phase_ms[4] = ms;
        return check_device_error(h->desc, h->stream);
    }
    std::vector<hipEvent_t> ev(4 * (size_t)n_sweeps + 2, nullptr);
    int rc = SW_OK;
    // timing-only events: no system-scope fence (cache write-back) at each one
    for (auto& e : ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            rc = fail(SW_EHIP, "hipEventCreate failed");
            break;
        }
    const Work w{h->d_desc, nullptr, h->g.ntiles, h->g.ty, h->stream, h->g.csum, h->g.xy};
    if (rc == SW_OK) rc = enqueue_sweeps(w, n_sweeps, h->g.cap != 0, h->d_desc, 1, nullptr, ev.data());
    if (rc == SW_OK) {
        h->done += n_sweeps;
        h->have_sweep = true;
        h->labels_resolved = false;
        if (hipEventSynchronize(ev.back()) != hipSuccess) rc = fail(SW_EHIP, "hipEventSynchronize failed");
    }
    // events of sweep k: 4k start, 4k+1 after the bond kernel, 4k+2 after the
    // labels, 4k+3 after the merge, 4k+4 after the flip (the next sweep's start)
    auto elapsed = [&](size_t a, size_t b, double& acc) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[a], ev[b]) != hipSuccess) return fail(SW_EHIP, "hipEventElapsedTime failed");
        acc += ms;
        return SW_OK;
    };
    for (uint32_t k = 0; rc == SW_OK && k < n_sweeps; ++k) {
        const size_t b = 4 * (size_t)k;
        rc = elapsed(b, b + 2, phase_ms[0]);
        if (rc == SW_OK) rc = elapsed(b + 2, b + 3, phase_ms[1]);
        if (rc == SW_OK) rc = elapsed(b + 3, b + 4, phase_ms[2]);
        if (rc == SW_OK) rc = elapsed(b, b + 1, phase_ms[4]);
    }
    if (rc == SW_OK) rc = elapsed(4 * (size_t)n_sweeps, ev.size() - 1, phase_ms[3]);
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc == SW_OK) rc = check_device_error(h->desc, h->stream);
    return rc;
}

int sw_sweeps_done(const sw_lattice* h, uint32_t* out)
{
    if (!h || !out) return fail(SW_EINVAL, "NULL argument");
    *out = h->done;
    return SW_OK;
}

int sw_measure_after(sw_lattice* h, void* read_stream, void* after_event, uint32_t first, uint32_t n,
                     int64_t* host_out)
{
    if (!h || !read_stream || (!host_out && n)) return fail(SW_EINVAL, "NULL argument");
    if (h->g.cap == 0) return fail(SW_ESTATE, "lattice was created with obs_capacity = 0");
    const uint64_t end = (uint64_t)first + n;
    const uint64_t lo = std::max<uint64_t>(h->first_obs, h->done > h->g.cap ? h->done - h->g.cap : 0);
    if (first < lo || end > h->done)
        return fail(SW_ESTATE, "sweeps [%u, %llu) not available (have [%llu, %u))", first,
                    (unsigned long long)end, (unsigned long long)lo, h->done);
    const hipStream_t rs = static_cast<hipStream_t>(read_stream);
    if (after_event) HIP_TRY(hipStreamWaitEvent(rs, static_cast<hipEvent_t>(after_event), 0));
    int rc = check_device_error(h->desc, rs);
    if (rc) return rc;
    return read_ring(h->desc, h->g.N, rs, first, n, host_out);
}

int sw_read_spins_after(sw_lattice* h, void* read_stream, void* after_event, uint8_t* host_out)
{
    if (!h || !read_stream || !host_out) return fail(SW_EINVAL, "NULL argument");
    if (h->g.xy) return fail(SW_EINVAL, "an XY lattice holds angles: read them with sw_xy_read_angles");
    const hipStream_t rs = static_cast<hipStream_t>(read_stream);
    if (after_event) HIP_TRY(hipStreamWaitEvent(rs, static_cast<hipEvent_t>(after_event), 0));
    HIP_TRY(hipMemcpyAsync(host_out, h->desc.s, h->g.N, hipMemcpyDeviceToHost, rs));
    return check_device_error(h->desc, rs);
}

int sw_measure(sw_lattice* h, uint32_t first, uint32_t n, int64_t* host_out)
{
    if (!h || (!host_out && n)) return fail(SW_EINVAL, "NULL argument");
    if (h->g.cap == 0) return fail(SW_ESTATE, "lattice was created with obs_capacity = 0");
    const uint64_t end = (uint64_t)first + n;
    const uint64_t lo = std::max<uint64_t>(h->first_obs, h->done > h->g.cap ? h->done - h->g.cap : 0);
    if (first < lo || end > h->done)
        return fail(SW_ESTATE, "sweeps [%u, %llu) not available (have [%llu, %u))", first,
                    (unsigned long long)end, (unsigned long long)lo, h->done);
    int rc = check_device_error(h->desc, h->stream);
    if (rc) return rc;
    return read_ring(h->desc, h->g.N, h->stream, first, n, host_out);
}

int sw_cluster_sums(sw_lattice* h, uint32_t first, uint32_t n, uint64_t* host_out)
{
    if (!h || (!host_out && n)) return fail(SW_EINVAL, "NULL argument");
    if (!h->g.csum) return fail(SW_ESTATE, "lattice was created without SW_CLUSTER_SUMS");
    const uint64_t end = (uint64_t)first + n;
    const uint64_t lo = std::max<uint64_t>(h->first_obs, h->done > h->g.cap ? h->done - h->g.cap : 0);
    if (first < lo || end > h->done)
        return fail(SW_ESTATE, "sweeps [%u, %llu) not available (have [%llu, %u))", first,
                    (unsigned long long)end, (unsigned long long)lo, h->done);
    int rc = check_device_error(h->desc, h->stream);
    if (rc) return rc;
    return read_ring(h->desc, h->g.N, h->stream, first, n, nullptr, host_out);
}

int sw_read_spins(sw_lattice* h, uint8_t* host_out)
{
    if (!h || !host_out) return fail(SW_EINVAL, "NULL argument");
    if (h->g.xy) return fail(SW_EINVAL, "an XY lattice holds angles: read them with sw_xy_read_angles");
    HIP_TRY(hipMemcpyAsync(host_out, h->desc.s, h->g.N, hipMemcpyDeviceToHost, h->stream));
    return check_device_error(h->desc, h->stream);
}

int sw_load_spins(sw_lattice* h, const uint8_t* host_in, uint32_t sweep)
{
    if (!h || !host_in) return fail(SW_EINVAL, "NULL argument");
    if (h->g.xy) return fail(SW_EINVAL, "an XY lattice holds angles: load them with sw_xy_load_angles");
    for (size_t i = 0; i < h->g.N; ++i)
        if (host_in[i] >= h->g.q) return fail(SW_EINVAL, "spin %u at site %zu is not below q", host_in[i], i);
    HIP_TRY(hipMemcpyAsync(h->desc.s, host_in, h->g.N, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->desc.counter, &sweep, sizeof sweep, hipMemcpyHostToDevice, h->stream));
    if (h->g.cap)
        HIP_TRY(hipMemsetAsync(h->desc.ring, 0, (size_t)ring_slots(h->g) * NCOPY * rec_stride(h->g) * 8, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->done = sweep;
    h->first_obs = sweep;
    h->have_sweep = false;
    h->labels_resolved = false;
    return SW_OK;
}

int sw_read_labels(sw_lattice* h, uint32_t* host_out)
{
    if (!h || !host_out) return fail(SW_EINVAL, "NULL argument");
    if (!h->have_sweep) return fail(SW_ESTATE, "no sweep since init / load");
    const Geometry& g = h->g;
    if (h->labels_resolved) {
        HIP_TRY(hipMemcpyAsync(host_out, h->desc.lab, g.N * 4, hipMemcpyDeviceToHost, h->stream));
        return check_device_error(h->desc, h->stream);
    }
    // resolved in bands of at most N/2 sites, below the tile labels they read
    const uint32_t band = std::max(1u, g.L / 2);
    for (uint32_t ya = 0; ya < g.L; ya += band) {
        const uint32_t yb = std::min(g.L, ya + band);
        HIP_TRY(launch_resolve(h->d_desc, 0, g.ntiles, g.ty, ya, yb, h->stream));
        HIP_TRY(hipMemcpyAsync(host_out + (size_t)ya * g.L, h->desc.lab, (size_t)(yb - ya) * g.L * 4,
                               hipMemcpyDeviceToHost, h->stream));
    }
    return check_device_error(h->desc, h->stream);
}

int sw_read_bonds(sw_lattice* h, uint64_t* host_out)
{
    if (!h || !host_out) return fail(SW_EINVAL, "NULL argument");
    if (!h->have_sweep) return fail(SW_ESTATE, "no sweep since init / load");
    const Geometry& g = h->g;
    std::vector<uint64_t> tiles((size_t)g.ntiles * 2 * g.ty);
    HIP_TRY(hipMemcpyAsync(tiles.data(), h->desc.bonds, tiles.size() * 8, hipMemcpyDeviceToHost, h->stream));
    const int rc = check_device_error(h->desc, h->stream);
    if (rc) return rc;
    // tile-major words -> two row-major planes of L rows by W words (W = tiles per row)
    for (uint32_t t = 0; t < g.ntiles; ++t) {
        const uint32_t ty = t / g.ntx, tx = t % g.ntx;
        const uint32_t y0 = ty * g.ty, rows = std::min(g.ty, g.L - y0);
        for (uint32_t p = 0; p < 2; ++p)
            for (uint32_t r = 0; r < rows; ++r)
                host_out[((size_t)p * g.L + y0 + r) * g.W + tx] = tiles[((size_t)t * 2 + p) * g.ty + r];
    }
    return SW_OK;
}

int sw_label_equivalence(sw_lattice* h, uint32_t* dev_labels, uint32_t* dev_flag, uint32_t max_iter,
                         uint32_t* iterations, double* ms)
{
    if (!h || !dev_labels || !dev_flag || !iterations) return fail(SW_EINVAL, "NULL argument");
    if (!h->have_sweep) return fail(SW_ESTATE, "no sweep since init / load");
    if (max_iter == 0) return fail(SW_EINVAL, "max_iter must be >= 1");
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    auto run = [&](uint32_t* it_out, float* ms_out) -> int {
        HIP_TRY(hipEventRecord(ev[0], h->stream));
        HIP_TRY(launch_le_init(h->d_desc, h->g.L, dev_labels, h->stream));
        uint32_t it = 0, flag = 1;
        // the host loop of the method: one scan + analysis pass, then read the flag
        while (flag && it < max_iter) {
            HIP_TRY(hipMemsetAsync(dev_flag, 0, sizeof(uint32_t), h->stream));
            HIP_TRY(launch_le_iteration(h->d_desc, h->g.L, h->g.ty, dev_labels, dev_flag, h->stream));
            HIP_TRY(hipMemcpyAsync(&flag, dev_flag, sizeof flag, hipMemcpyDeviceToHost, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
            ++it;
        }
        HIP_TRY(hipEventRecord(ev[1], h->stream));
        HIP_TRY(hipEventSynchronize(ev[1]));
        HIP_TRY(hipEventElapsedTime(ms_out, ev[0], ev[1]));
        if (flag) return fail(SW_ECONVERGE, "label equivalence still changing after %u iterations", max_iter);
        *it_out = it;
        return SW_OK;
    };
    uint32_t it = 0;
    float elapsed = 0.f;
    int rc = run(&it, &elapsed);
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc) return rc;
    *iterations = it;
    if (ms) *ms = elapsed;
    return check_device_error(h->desc, h->stream);
}

int sw_destroy(sw_lattice* h)
{
    if (!h) return SW_OK;
    h->graphs.clear();
    delete h;
    return SW_OK;
}

int sw_derived(uint32_t L, uint32_t q, const int64_t* row, double* out)
{
    if (!row || !out) return fail(SW_EINVAL, "NULL argument");
    if (L < 2 || L > 65536 || q < 2 || q > 255) return fail(SW_EINVAL, "L = %u or q = %u out of range", L, q);
    const int64_t N = (int64_t)L * L;
    int64_t total = 0, most = 0;
    for (uint32_t c = 0; c < q; ++c) {
        const int64_t n = row[2 + c];
        if (n < 0 || n > N) return fail(SW_EINVAL, "count of state %u is %lld", c, (long long)n);
        total += n;
        most = std::max(most, n);
    }
    if (total != N) return fail(SW_EINVAL, "state counts add up to %lld, not N = %lld", (long long)total, (long long)N);
    const double Nd = (double)N;
    out[0] = (double)row[0] / Nd;                              // energy per site (units of J)
    out[1] = ((double)q * ((double)most / Nd) - 1.0) / (double)(q - 1);   // Potts order parameter
    out[2] = (q == 2) ? (double)(row[2] - row[3]) : 0.0;         // Ising magnetisation
    return SW_OK;
}

// ------------------------------------------------------------------ XY model

size_t sw_xy_workspace_bytes(const sw_xy_params* p)
{
    Geometry g;
    if (check_xy_params(p, &g) != SW_OK) return 0;
    return carve(g).total;
}

int sw_xy_init(const sw_xy_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, sw_lattice** out)
{
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    Geometry g;
    const int rc = check_xy_params(p, &g);
    if (rc) return rc;
    return create_lattice(g, p->seed, p->init, dev_ws, ws_bytes, hip_stream, out);
}

int sw_xy_read_angles(sw_lattice* h, uint32_t* host_out)
{
    if (!h || !host_out) return fail(SW_EINVAL, "NULL argument");
    if (!h->g.xy) return fail(SW_EINVAL, "not an XY lattice");
    HIP_TRY(hipMemcpyAsync(host_out, h->desc.ang, h->g.N * 4, hipMemcpyDeviceToHost, h->stream));
    return check_device_error(h->desc, h->stream);
}

int sw_xy_load_angles(sw_lattice* h, const uint32_t* host_in, uint32_t sweep)
{
    if (!h || !host_in) return fail(SW_EINVAL, "NULL argument");
    if (!h->g.xy) return fail(SW_EINVAL, "not an XY lattice");
    HIP_TRY(hipMemcpyAsync(h->desc.ang, host_in, h->g.N * 4, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->desc.counter, &sweep, sizeof sweep, hipMemcpyHostToDevice, h->stream));
    if (h->g.cap)
        HIP_TRY(hipMemsetAsync(h->desc.ring, 0, (size_t)ring_slots(h->g) * NCOPY * rec_stride(h->g) * 8, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->done = sweep;
    h->first_obs = sweep;
    h->have_sweep = false;
    h->labels_resolved = false;
    return SW_OK;
}

int sw_xy_derived(uint32_t L, double K, const int64_t* row, double* out)
{
    if (!row || !out) return fail(SW_EINVAL, "NULL argument");
    if (L < 2 || L > 65536) return fail(SW_EINVAL, "L = %u outside 2..65536", L);
    if (std::isnan(K) || K < 0) return fail(SW_EINVAL, "K must be >= 0 (got %g)", K);
    const double N = (double)L * (double)L;
    const double lim = N * 1073741824.0;   // |a sum| <= N in units of 2^-30
    for (int j = 1; j < (int)XY_WORDS; ++j)
        if (std::fabs((double)row[j]) > lim) return fail(SW_EINVAL, "word %d of the row exceeds N", j);
    const double u = 1.0 / 1073741824.0;   // 2^-30
    const double ex = row[1] * u, ey = row[2] * u, ix = row[3] * u, iy = row[4] * u, mx = row[5] * u, my = row[6] * u;
    out[0] = -(ex + ey) / N;                                     // energy per site (units of J)
    out[1] = (mx * mx + my * my) / (N * N);                      // squared magnetisation per site
    out[2] = (0.5 * (ex + ey) - K * 0.5 * (ix * ix + iy * iy)) / N;   // helicity estimator (units of J)
    return SW_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batched
// Replicas live one after another in the workspace, each laid out like a plain
// lattice; a header in front holds the descriptor table, the work map (tile
// list of the replicas being swept, largest sweep count first) and per-replica
// sweep counts.
struct sw_batch {
    uint32_t n;
    uint32_t ty;
    hipStream_t stream;
    char* base;
    std::vector<sw_params> p;
    std::vector<Geometry> g;
    std::vector<size_t> off;        // byte offset of replica r's slice
    std::vector<Carve> c;
    std::vector<LatDesc> desc;
    std::vector<uint32_t> done, first_obs;
    LatDesc* d_descs;
    WorkItem* d_map;
    uint32_t* d_n;
    size_t total_tiles;
    std::vector<WorkItem> h_map;    // host copy of the last uploaded map
    std::vector<uint32_t> h_n;
    std::vector<uint32_t> map_order;  // replica order of the uploaded map
    StepGraphs steps;                            // captured sweeps of every replica (sweep_all)
    bool csum = false;                           // some replica measures cluster-size sums
    // replicas swept whole (k_whole): device list, L <= 64 first, then the rest
    uint32_t* d_list = nullptr;
    uint32_t n_whole64 = 0, n_whole128 = 0;
    size_t tile_tiles = 0;                       // tiles of the replicas swept by tiles
};

namespace {

struct BatchLayout {
    size_t descs, map, nvec, list, header;
    std::vector<size_t> off;
    std::vector<Geometry> g;
    std::vector<Carve> c;
    size_t total_tiles, total;
    uint32_t ty;
};

int batch_layout(const sw_params* params, uint32_t n, BatchLayout* out)
{
    if (!params || n == 0) return fail(SW_EINVAL, "need at least one replica");
    BatchLayout b{};
    b.g.resize(n);
    b.c.resize(n);
    b.off.resize(n);
    b.total_tiles = 0;
    for (uint32_t r = 0; r < n; ++r) {
        int rc = check_params(&params[r], &b.g[r]);
        if (rc) return fail(rc, "replica %u: %s", r, g_err.c_str());
        if (r && b.g[r].ty != b.g[0].ty) return fail(SW_EINVAL, "all replicas need the same tile_rows");
        b.c[r] = carve(b.g[r]);
        b.total_tiles += b.g[r].ntiles;
    }
    if (b.total_tiles >= 0xFFFFFFFFull) return fail(SW_EINVAL, "too many tiles in one batch");
    b.ty = b.g[0].ty;
    size_t off = 0;
    b.descs = off;
    off = align_up(off + sizeof(LatDesc) * n);
    b.map = off;
    off = align_up(off + sizeof(WorkItem) * b.total_tiles);
    b.nvec = off;
    off = align_up(off + sizeof(uint32_t) * n);
    b.list = off;
    off = align_up(off + sizeof(uint32_t) * n);
    b.header = off;
    for (uint32_t r = 0; r < n; ++r) {
        b.off[r] = off;
        off = align_up(off + b.c[r].total);
    }
    b.total = off;
    *out = std::move(b);
    return SW_OK;
}

// Upload the tile list of the replicas with n_each[r] > 0, largest count first,
// so that the replicas still sweeping at step k are a prefix of the list.
// Returns, through prefix[k], the number of work items active at step k.
int upload_map(sw_batch* b, const uint32_t* n_each, uint32_t kmax, std::vector<uint32_t>* prefix)
{
    std::vector<uint32_t> order;
    for (uint32_t r = 0; r < b->n; ++r)
        if (n_each[r] && !b->g[r].whole) order.push_back(r);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) { return n_each[a] > n_each[c]; });
    if (order != b->map_order || b->h_map.empty()) {
        b->h_map.clear();
        for (uint32_t r : order)
            for (uint32_t t = 0; t < b->g[r].ntiles; ++t) b->h_map.push_back({r, t});
        if (!b->h_map.empty())
            HIP_TRY(hipMemcpyAsync(b->d_map, b->h_map.data(), b->h_map.size() * sizeof(WorkItem),
                                   hipMemcpyHostToDevice, b->stream));
        b->map_order = order;
    }
    prefix->assign(kmax, 0);
    size_t acc = 0;
    // replicas sorted by count descending: at step k the active ones are those with n > k
    std::vector<size_t> ends;
    for (uint32_t r : order) {
        acc += b->g[r].ntiles;
        ends.push_back(acc);
    }
    for (uint32_t k = 0; k < kmax; ++k) {
        size_t m = 0;
        for (size_t i = 0; i < order.size(); ++i)
            if (n_each[order[i]] > k) m = ends[i];
        (*prefix)[k] = (uint32_t)m;
    }
    return SW_OK;
}

// The replicas swept whole: n_each[r] (or n_uniform) sweeps from counter + k0,
// counters left for the caller to advance.
int batch_whole(sw_batch* b, uint32_t k0, uint32_t n_uniform, const uint32_t* d_n_each)
{
    HIP_TRY(launch_whole(b->d_descs, b->d_list, b->n_whole64, 64, k0, n_uniform, d_n_each, 2u, b->ty, b->stream));
    HIP_TRY(launch_whole(b->d_descs, b->d_list + b->n_whole64, b->n_whole128, WHOLE_LMAX, k0, n_uniform, d_n_each, 2u,
                         b->ty, b->stream));
    return SW_OK;
}

int batch_enqueue(sw_batch* b, const uint32_t* n_each)
{
    uint32_t kmax = 0, kall = 0;
    for (uint32_t r = 0; r < b->n; ++r) {
        kall = std::max(kall, n_each[r]);
        if (!b->g[r].whole) kmax = std::max(kmax, n_each[r]);
    }
    if (kall == 0) return SW_OK;
    b->h_n.assign(n_each, n_each + b->n);
    HIP_TRY(hipMemcpyAsync(b->d_n, b->h_n.data(), b->n * sizeof(uint32_t), hipMemcpyHostToDevice, b->stream));
    int rc = batch_whole(b, 0, 0, b->d_n);
    if (rc) return rc;
    std::vector<uint32_t> prefix;
    if (kmax) {
        rc = upload_map(b, n_each, kmax, &prefix);
        if (rc) return rc;
    }
    for (uint32_t k = 0; k < kmax; ++k) {
        const Work w{b->d_descs, b->d_map, prefix[k], b->ty, b->stream, b->csum};
        HIP_TRY(launch_bond_label(w, k, k > 0 ? 1u : 0u));
        HIP_TRY(launch_merge(w));
        HIP_TRY(launch_flip(w, k));
        if (w.cluster) HIP_TRY(launch_cluster_sums(w, k));
    }
    if (kmax) {
        const Work w0{b->d_descs, b->d_map, prefix[0], b->ty, b->stream};
        HIP_TRY(launch_measure_each(w0, b->d_n));
    }
    HIP_TRY(launch_bump(b->d_descs, b->n, b->d_n, 0, b->stream));
    return SW_OK;
}

int batch_check(const sw_batch* b, uint32_t replica)
{
    if (!b) return fail(SW_EINVAL, "batch is NULL");
    if (replica >= b->n) return fail(SW_EINVAL, "replica %u out of range (%u replicas)", replica, b->n);
    return SW_OK;
}

}  // namespace

extern "C" {

int sw_batch_workspace_bytes(const sw_params* params, uint32_t n, size_t* bytes)
{
    if (!bytes) return fail(SW_EINVAL, "bytes is NULL");
    BatchLayout b;
    int rc = batch_layout(params, n, &b);
    if (rc) return rc;
    *bytes = b.total;
    return SW_OK;
}

int sw_batch_init(const sw_params* params, uint32_t n, void* dev_ws, size_t ws_bytes, void* hip_stream,
                  sw_batch** out)
{
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    BatchLayout lay;
    int rc = batch_layout(params, n, &lay);
    if (rc) return rc;
    if (!dev_ws || ((uintptr_t)dev_ws % ALIGN) != 0)
        return fail(SW_ESPACE, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < lay.total) return fail(SW_ESPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);
    sw_batch* b = new (std::nothrow) sw_batch();
    if (!b) return fail(SW_EINVAL, "out of host memory");
    b->n = n;
    b->ty = lay.ty;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->base = static_cast<char*>(dev_ws);
    b->p.assign(params, params + n);
    b->g = lay.g;
    b->c = lay.c;
    b->off = lay.off;
    b->total_tiles = lay.total_tiles;
    b->done.assign(n, 0);
    b->first_obs.assign(n, 0);
    b->d_descs = reinterpret_cast<LatDesc*>(b->base + lay.descs);
    b->d_map = reinterpret_cast<WorkItem*>(b->base + lay.map);
    b->d_n = reinterpret_cast<uint32_t*>(b->base + lay.nvec);
    b->d_list = reinterpret_cast<uint32_t*>(b->base + lay.list);
    std::vector<uint32_t> list;
    for (uint32_t r = 0; r < n; ++r)
        if (lay.g[r].whole && lay.g[r].L <= 64) list.push_back(r);
    b->n_whole64 = (uint32_t)list.size();
    for (uint32_t r = 0; r < n; ++r)
        if (lay.g[r].whole && lay.g[r].L > 64) list.push_back(r);
    b->n_whole128 = (uint32_t)list.size() - b->n_whole64;
    for (uint32_t r = 0; r < n; ++r)
        if (!lay.g[r].whole) b->tile_tiles += lay.g[r].ntiles;
    b->desc.resize(n);
    for (uint32_t r = 0; r < n; ++r) b->csum = b->csum || b->g[r].csum;
    for (uint32_t r = 0; r < n; ++r) {
        b->desc[r] = make_desc(b->g[r], params[r].seed, b->base + b->off[r], b->c[r]);
        if (!division_ok(b->g[r].L, b->desc[r].magic, b->desc[r].shift)) {
            delete b;
            return fail(SW_EINVAL, "internal: division by L self-check failed");
        }
    }
    auto run = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(b->d_descs, b->desc.data(), sizeof(LatDesc) * n, hipMemcpyHostToDevice, b->stream));
        if (!list.empty())
            HIP_TRY(hipMemcpyAsync(b->d_list, list.data(), list.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                   b->stream));
        for (uint32_t r = 0; r < n; ++r) {
            char* base = b->base + b->off[r];
            HIP_TRY(hipMemsetAsync(base + b->c[r].state, 0, sizeof(DevState), b->stream));
            if (b->g[r].cap)
                HIP_TRY(hipMemsetAsync(base + b->c[r].ring, 0,
                                       (size_t)ring_slots(b->g[r]) * NCOPY * ring_stride(b->g[r].q) * 8, b->stream));
            if (b->g[r].csum)
                HIP_TRY(hipMemsetAsync(base + b->c[r].csize, 0, (size_t)b->g[r].ntiles * nslot(b->g[r].ty) * 8,
                                       b->stream));
            if (params[r].init) HIP_TRY(launch_init(b->d_descs, r, b->g[r].N, 1u, b->stream));
            else HIP_TRY(hipMemsetAsync(b->desc[r].s, 0, b->g[r].N, b->stream));
        }
        HIP_TRY(hipStreamSynchronize(b->stream));
        return SW_OK;
    };
    rc = run();
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return SW_OK;
}

int sw_batch_sweep(sw_batch* b, const uint32_t* n_sweeps)
{
    if (!b || !n_sweeps) return fail(SW_EINVAL, "NULL argument");
    for (uint32_t r = 0; r < b->n; ++r)
        if ((uint64_t)b->done[r] + n_sweeps[r] > 0xFFFFFFFFull)
            return fail(SW_ESTATE, "replica %u: sweep counter would overflow", r);
    int rc = batch_enqueue(b, n_sweeps);
    if (rc) return rc;
    for (uint32_t r = 0; r < b->n; ++r) b->done[r] += n_sweeps[r];
    return SW_OK;
}

int sw_batch_sweep_all(sw_batch* b, uint32_t n_sweeps)
{
    if (!b) return fail(SW_EINVAL, "batch is NULL");
    if (n_sweeps == 0) return SW_OK;
    for (uint32_t r = 0; r < b->n; ++r)
        if ((uint64_t)b->done[r] + n_sweeps > 0xFFFFFFFFull)
            return fail(SW_ESTATE, "replica %u: sweep counter would overflow", r);
    std::vector<uint32_t> all(b->n, n_sweeps);
    if (b->stream == nullptr) {
        // the legacy default stream cannot be captured: launch directly
        const int rc = batch_enqueue(b, all.data());
        if (rc) return rc;
        for (uint32_t r = 0; r < b->n; ++r) b->done[r] += n_sweeps;
        return SW_OK;
    }
    if (b->n_whole64 + b->n_whole128) {
        // the replicas swept whole first, in launches of at most WHOLE_CHUNK
        // sweeps; their counters advance with everyone's below
        for (uint32_t done = 0; done < n_sweeps;) {
            const uint32_t k = std::min(WHOLE_CHUNK, n_sweeps - done);
            const int rc = batch_whole(b, done, k, nullptr);
            if (rc) return rc;
            done += k;
        }
        if (b->tile_tiles == 0) {
            HIP_TRY(launch_bump(b->d_descs, b->n, nullptr, n_sweeps, b->stream));
            for (uint32_t r = 0; r < b->n; ++r) b->done[r] += n_sweeps;
            return SW_OK;
        }
    }
    // the captured steps bake in the work map of every replica swept by
    // tiles; make sure it is the one uploaded
    std::vector<uint32_t> order;
    for (uint32_t r = 0; r < b->n; ++r)
        if (!b->g[r].whole) order.push_back(r);
    if (b->map_order != order || b->h_map.empty()) {
        std::vector<uint32_t> prefix;
        int rc = upload_map(b, all.data(), 1, &prefix);
        if (rc) return rc;
    }
    const Work w{b->d_descs, b->d_map, (uint32_t)b->tile_tiles, b->ty, b->stream, b->csum};
    // replicas without a ring skip the measurements inside the kernels
    const int rc = run_steps(b->steps, w, n_sweeps, true, b->d_descs, b->n);
    if (rc) return rc;
    for (uint32_t r = 0; r < b->n; ++r) b->done[r] += n_sweeps;
    return SW_OK;
}

int sw_batch_measure(sw_batch* b, uint32_t replica, uint32_t first, uint32_t n, int64_t* host_out)
{
    int rc = batch_check(b, replica);
    if (rc) return rc;
    if (!host_out && n) return fail(SW_EINVAL, "host_out is NULL");
    const Geometry& g = b->g[replica];
    if (g.cap == 0) return fail(SW_ESTATE, "replica %u was created with obs_capacity = 0", replica);
    const uint64_t end = (uint64_t)first + n;
    const uint32_t done = b->done[replica];
    const uint64_t lo = std::max<uint64_t>(b->first_obs[replica], done > g.cap ? done - g.cap : 0);
    if (first < lo || end > done) return fail(SW_ESTATE, "sweeps [%u, %llu) not available", first, (unsigned long long)end);
    rc = check_device_error(b->desc[replica], b->stream);
    if (rc) return rc;
    return read_ring(b->desc[replica], g.N, b->stream, first, n, host_out);
}

int sw_batch_cluster_sums(sw_batch* b, uint32_t replica, uint32_t first, uint32_t n, uint64_t* host_out)
{
    int rc = batch_check(b, replica);
    if (rc) return rc;
    if (!host_out && n) return fail(SW_EINVAL, "host_out is NULL");
    const Geometry& g = b->g[replica];
    if (!g.csum) return fail(SW_ESTATE, "replica %u was created without SW_CLUSTER_SUMS", replica);
    const uint64_t end = (uint64_t)first + n;
    const uint32_t done = b->done[replica];
    const uint64_t lo = std::max<uint64_t>(b->first_obs[replica], done > g.cap ? done - g.cap : 0);
    if (first < lo || end > done) return fail(SW_ESTATE, "sweeps [%u, %llu) not available", first, (unsigned long long)end);
    rc = check_device_error(b->desc[replica], b->stream);
    if (rc) return rc;
    return read_ring(b->desc[replica], g.N, b->stream, first, n, nullptr, host_out);
}

int sw_batch_read_spins(sw_batch* b, uint32_t replica, uint8_t* host_out)
{
    int rc = batch_check(b, replica);
    if (rc) return rc;
    if (!host_out) return fail(SW_EINVAL, "host_out is NULL");
    HIP_TRY(hipMemcpyAsync(host_out, b->desc[replica].s, b->g[replica].N, hipMemcpyDeviceToHost, b->stream));
    return check_device_error(b->desc[replica], b->stream);
}

int sw_batch_sweeps_done(const sw_batch* b, uint32_t replica, uint32_t* out)
{
    int rc = batch_check(b, replica);
    if (rc) return rc;
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = b->done[replica];
    return SW_OK;
}

int sw_batch_destroy(sw_batch* b)
{
    if (!b) return SW_OK;
    b->steps.clear();
    delete b;
    return SW_OK;
}

int sw_batch_autotune(const sw_params* params, uint32_t n, const uint32_t* candidates, uint32_t n_candidates,
                      uint32_t sweeps, void* dev_ws, size_t ws_bytes, void* hip_stream, uint32_t* tile_rows,
                      double* ms_per_sweep)
{
    if (!params || !candidates || !tile_rows) return fail(SW_EINVAL, "NULL argument");
    if (n == 0) return fail(SW_EINVAL, "need at least one replica");
    if (n_candidates == 0 || n_candidates > 8) return fail(SW_EINVAL, "need 1 to 8 candidate tile heights");
    if (sweeps == 0 || sweeps > 4096) return fail(SW_EINVAL, "time 1 to 4096 sweeps per candidate");
    std::vector<sw_params> p(params, params + n);
    // every candidate is checked (and its workspace sized) before the first launch
    for (uint32_t c = 0; c < n_candidates; ++c) {
        const uint32_t ty = candidates[c];
        if (ty != 0 && ty != SW_TILE_WHOLE && ty != 32 && ty != 64 && ty != 128)
            return fail(SW_EINVAL, "candidate tile height %u is not 0, SW_TILE_WHOLE, 32, 64 or 128", ty);
        for (auto& pr : p) pr.tile_rows = ty;
        size_t need = 0;
        const int rc = sw_batch_workspace_bytes(p.data(), n, &need);
        if (rc) return rc;
        if (!dev_ws || ((uintptr_t)dev_ws % ALIGN) != 0)
            return fail(SW_ESPACE, "workspace must be a 256-byte aligned device pointer");
        if (ws_bytes < need) return fail(SW_ESPACE, "tile height %u needs %zu workspace bytes, have %zu", ty, need, ws_bytes);
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    int rc = SW_OK;
    uint32_t best = 0;
    double best_ms = 0.0;
    for (uint32_t c = 0; c < n_candidates && rc == SW_OK; ++c) {
        for (auto& pr : p) pr.tile_rows = candidates[c];
        sw_batch* b = nullptr;
        rc = sw_batch_init(p.data(), n, dev_ws, ws_bytes, hip_stream, &b);
        if (rc) break;
        // one untimed pass (graph capture, caches), then the timed one
        rc = sw_batch_sweep_all(b, sweeps);
        if (rc == SW_OK && hipEventRecord(ev[0], b->stream) != hipSuccess) rc = fail(SW_EHIP, "hipEventRecord failed");
        if (rc == SW_OK) rc = sw_batch_sweep_all(b, sweeps);
        if (rc == SW_OK && hipEventRecord(ev[1], b->stream) != hipSuccess) rc = fail(SW_EHIP, "hipEventRecord failed");
        if (rc == SW_OK && hipEventSynchronize(ev[1]) != hipSuccess) rc = fail(SW_EHIP, "hipEventSynchronize failed");
        float ms = 0.f;
        if (rc == SW_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess)
            rc = fail(SW_EHIP, "hipEventElapsedTime failed");
        for (uint32_t r = 0; rc == SW_OK && r < n; ++r) rc = check_device_error(b->desc[r], b->stream);
        (void)sw_batch_destroy(b);
        if (rc) break;
        const double per = (double)ms / sweeps;
        if (ms_per_sweep) ms_per_sweep[c] = per;
        if (c == 0 || per < best_ms) {
            best = candidates[c];
            best_ms = per;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc == SW_OK) *tile_rows = best;
    return rc;
}

}  // extern "C"

// -------------------------------------------------------------------- groups
// A group sweeps any set of separately initialised lattices (same tile height,
// same stream) with one launch per phase: the continuous-batching primitive,
// where lattices join and leave between calls.  Its device scratch (descriptor
// table, work map, per-lattice sweep counts) comes from the caller's workspace.
struct sw_group {
    uint32_t max_lat;
    uint64_t max_tiles;
    uint32_t ty;
    hipStream_t stream;
    LatDesc* d_descs;
    WorkItem* d_map;
    uint32_t* d_n;
    std::vector<LatDesc> h_desc;
    std::vector<WorkItem> h_map;
    std::vector<uint32_t> h_n;
};

namespace {

struct GroupLayout {
    size_t descs, map, nvec, total;
};

GroupLayout group_layout(uint32_t max_lat, uint64_t max_tiles)
{
    GroupLayout g{};
    size_t off = 0;
    g.descs = off;
    off = align_up(off + sizeof(LatDesc) * max_lat);
    g.map = off;
    off = align_up(off + sizeof(WorkItem) * max_tiles);
    g.nvec = off;
    off = align_up(off + sizeof(uint32_t) * max_lat);
    g.total = off;
    return g;
}

}  // namespace

extern "C" {

int sw_tile_count(const sw_params* p, uint32_t* tiles)
{
    if (!tiles) return fail(SW_EINVAL, "tiles is NULL");
    Geometry g;
    const int rc = check_params(p, &g);
    if (rc) return rc;
    *tiles = g.ntiles;
    return SW_OK;
}

int sw_group_workspace_bytes(uint32_t max_lattices, uint64_t max_tiles, size_t* bytes)
{
    if (!bytes) return fail(SW_EINVAL, "bytes is NULL");
    if (max_lattices == 0 || max_tiles == 0 || max_tiles >= 0xFFFFFFFFull)
        return fail(SW_EINVAL, "need 1 <= max_lattices and 1 <= max_tiles < 2^32");
    *bytes = group_layout(max_lattices, max_tiles).total;
    return SW_OK;
}

int sw_group_init(uint32_t max_lattices, uint64_t max_tiles, uint32_t tile_rows, void* dev_ws, size_t ws_bytes,
                  void* hip_stream, sw_group** out)
{
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    int rc = sw_group_workspace_bytes(max_lattices, max_tiles, &need);
    if (rc) return rc;
    const uint32_t ty = tile_rows ? tile_rows : DEFAULT_TY;
    if (ty != 32 && ty != 64 && ty != 128) return fail(SW_EINVAL, "tile_rows must be 0, 32, 64 or 128");
    if (!dev_ws || ((uintptr_t)dev_ws % ALIGN) != 0)
        return fail(SW_ESPACE, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < need) return fail(SW_ESPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    sw_group* g = new (std::nothrow) sw_group();
    if (!g) return fail(SW_EINVAL, "out of host memory");
    const GroupLayout lay = group_layout(max_lattices, max_tiles);
    char* base = static_cast<char*>(dev_ws);
    g->max_lat = max_lattices;
    g->max_tiles = max_tiles;
    g->ty = ty;
    g->stream = static_cast<hipStream_t>(hip_stream);
    g->d_descs = reinterpret_cast<LatDesc*>(base + lay.descs);
    g->d_map = reinterpret_cast<WorkItem*>(base + lay.map);
    g->d_n = reinterpret_cast<uint32_t*>(base + lay.nvec);
    *out = g;
    return SW_OK;
}

int sw_group_sweep(sw_group* g, sw_lattice* const* lats, const uint32_t* n_sweeps, uint32_t n)
{
    if (!g || (n && (!lats || !n_sweeps))) return fail(SW_EINVAL, "NULL argument");
    if (n > g->max_lat) return fail(SW_EINVAL, "%u lattices exceed the group's %u", n, g->max_lat);
    uint64_t tiles = 0;
    uint32_t kmax = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const sw_lattice* h = lats[i];
        if (!h) return fail(SW_EINVAL, "lattice %u is NULL", i);
        if (h->g.xy) return fail(SW_EINVAL, "lattice %u is an XY lattice; groups step Potts lattices", i);
        if (h->g.ty != g->ty) return fail(SW_EINVAL, "lattice %u has tile_rows %u, group %u", i, h->g.ty, g->ty);
        if (h->stream != g->stream) return fail(SW_EINVAL, "lattice %u is bound to another stream", i);
        if ((uint64_t)h->done + n_sweeps[i] > 0xFFFFFFFFull)
            return fail(SW_ESTATE, "lattice %u: sweep counter would overflow", i);
        for (uint32_t j = 0; j < i; ++j)
            if (lats[j] == h) return fail(SW_EINVAL, "lattice %u appears twice", i);
        if (n_sweeps[i]) tiles += h->g.ntiles;
        kmax = std::max(kmax, n_sweeps[i]);
    }
    bool csum = false;
    for (uint32_t i = 0; i < n; ++i) csum = csum || (n_sweeps[i] && lats[i]->g.csum);
    if (tiles > g->max_tiles) return fail(SW_EINVAL, "%llu tiles exceed the group's %llu",
                                          (unsigned long long)tiles, (unsigned long long)g->max_tiles);
    if (kmax == 0) return SW_OK;
    // work map: tiles of the lattices still sweeping at step k form a prefix
    std::vector<uint32_t> order;
    for (uint32_t i = 0; i < n; ++i)
        if (n_sweeps[i]) order.push_back(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t c) { return n_sweeps[a] > n_sweeps[c]; });
    g->h_desc.resize(n);
    g->h_n.assign(n_sweeps, n_sweeps + n);
    g->h_map.clear();
    for (uint32_t i = 0; i < n; ++i) g->h_desc[i] = lats[i]->desc;
    std::vector<uint32_t> ends;
    for (uint32_t i : order) {
        for (uint32_t t = 0; t < lats[i]->g.ntiles; ++t) g->h_map.push_back({i, t});
        ends.push_back((uint32_t)g->h_map.size());
    }
    HIP_TRY(hipMemcpyAsync(g->d_descs, g->h_desc.data(), sizeof(LatDesc) * n, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipMemcpyAsync(g->d_map, g->h_map.data(), sizeof(WorkItem) * g->h_map.size(), hipMemcpyHostToDevice,
                           g->stream));
    HIP_TRY(hipMemcpyAsync(g->d_n, g->h_n.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, g->stream));
    size_t pos = order.size();
    for (uint32_t k = 0; k < kmax; ++k) {
        while (pos > 0 && n_sweeps[order[pos - 1]] <= k) --pos;
        const Work w{g->d_descs, g->d_map, pos ? ends[pos - 1] : 0u, g->ty, g->stream, csum};
        HIP_TRY(launch_bond_label(w, k, k > 0 ? 1u : 0u));
        HIP_TRY(launch_merge(w));
        HIP_TRY(launch_flip(w, k));
        if (w.cluster) HIP_TRY(launch_cluster_sums(w, k));
    }
    const Work w0{g->d_descs, g->d_map, ends.back(), g->ty, g->stream};
    HIP_TRY(launch_measure_each(w0, g->d_n));
    HIP_TRY(launch_bump(g->d_descs, n, g->d_n, 0, g->stream));
    for (uint32_t i = 0; i < n; ++i)
        if (n_sweeps[i]) {
            lats[i]->done += n_sweeps[i];
            lats[i]->have_sweep = true;
            lats[i]->labels_resolved = false;
        }
    return SW_OK;
}

int sw_group_destroy(sw_group* g)
{
    delete g;
    return SW_OK;
}

}  // extern "C"

// ------------------------------------------------------- no-allocation entry
// For callers that cannot allocate (graph capture, tight serving loops): the
// labels, bond words, edge records, ring, state and descriptor of one lattice
// live in a fixed array of device memory that the library owns (one copy per
// GPU, held until the process ends); the caller passes only the spins and the
// observable rows.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[SW_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch;   // device -> address of that device's copy of scratch

int scratch_address(hipStream_t stream, char** out)
{
    int dev = 0;
    if (stream) HIP_TRY(hipStreamGetDevice(stream, &dev));
    else HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) return fail(SW_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        it = g_scratch.emplace(dev, static_cast<char*>(ptr)).first;
    }
    *out = it->second;
    return SW_OK;
}

// Ring slots of the no-allocation form: a record is read out right after it
// is complete, and the flip clears the slot after next ahead of time.
constexpr uint32_t STATIC_SLOTS = 3;

struct StaticCarve {
    size_t state, desc, lab, bonds, edges, nodes, ring, total;
};

StaticCarve carve_static(const Geometry& g, bool measure)
{
    StaticCarve c{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    c.state = take(sizeof(DevState));
    c.desc = take(sizeof(LatDesc));
    c.lab = take(g.N * 4);
    c.bonds = take((size_t)g.ntiles * 2 * g.ty * 8);
    c.edges = take((size_t)g.ntiles * edge_words(g.ty) * 4);
    c.nodes = take((size_t)g.ntiles * nslot(g.ty) * 8);
    c.ring = take(measure ? (size_t)STATIC_SLOTS * NCOPY * ring_stride(g.q) * 8 : 0);
    c.total = off;
    return c;
}

}  // namespace

extern "C" int sw_sweep_static(const sw_params* p, uint8_t* dev_spins, uint32_t first_sweep, uint32_t n_sweeps,
                               int64_t* dev_obs, uint32_t* dev_status, void* hip_stream)
{
    Geometry g;
    int rc = check_params(p, &g);
    if (rc) return rc;
    if (!dev_spins) return fail(SW_EINVAL, "dev_spins is NULL");
    if (g.csum) return fail(SW_EINVAL, "cluster sums are not measured by this entry point");
    if ((uint64_t)first_sweep + n_sweeps > 0xFFFFFFFFull) return fail(SW_ESTATE, "sweep counter would overflow");
    const bool measure = dev_obs != nullptr;
    const StaticCarve c = carve_static(g, measure);
    if (c.total > SW_STATIC_SCRATCH_BYTES)
        return fail(SW_ESPACE, "L = %u, tile_rows = %u needs %zu bytes of scratch; the library holds %u (L <= 2048 fits)",
                    g.L, g.ty, c.total, (unsigned)SW_STATIC_SCRATCH_BYTES);
    if (n_sweeps == 0) return SW_OK;
    const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    char* base = nullptr;
    rc = scratch_address(stream, &base);
    if (rc) return rc;

    // the descriptor: the caller's spins, everything else in scratch
    sw_params q = *p;
    q.obs_capacity = measure ? STATIC_SLOTS - 1 : 0;
    Carve pc{};
    pc.state = c.state;
    pc.desc = c.desc;
    pc.lab = c.lab;
    pc.bonds = c.bonds;
    pc.edges = c.edges;
    pc.nodes = c.nodes;
    pc.ring = c.ring;
    pc.obs = c.ring;   // no read staging in this form
    Geometry gq = g;
    gq.cap = q.obs_capacity;
    LatDesc d = make_desc(gq, q.seed, base, pc);
    if (!division_ok(g.L, d.magic, d.shift)) return fail(SW_EINVAL, "internal: division by L self-check failed");
    d.s = dev_spins;
    d.obs = nullptr;
    DevState* st = reinterpret_cast<DevState*>(base + c.state);
    LatDesc* d_desc = reinterpret_cast<LatDesc*>(base + c.desc);
    int64_t* ring = measure ? reinterpret_cast<int64_t*>(base + c.ring) : nullptr;
    const uint32_t ring_words = measure ? STATIC_SLOTS * NCOPY * ring_stride(g.q) : 0;
    const uint32_t W = 2 + g.q;

    HIP_TRY(launch_static_setup(d, d_desc, st, first_sweep, ring, ring_words, stream));
    const Work w{d_desc, nullptr, g.ntiles, g.ty, stream};
    for (uint32_t k = 0; k < n_sweeps; ++k) {
        HIP_TRY(launch_bond_label(w, k, (measure && k > 0) ? 1u : 0u));
        // the record of sweep k - 1 is complete once the bonds of sweep k are drawn
        if (measure && k > 0)
            HIP_TRY(launch_emit_row(ring, STATIC_SLOTS, first_sweep + k - 1, g.q, g.N, dev_obs + (size_t)(k - 1) * W,
                                    nullptr, nullptr, stream));
        HIP_TRY(launch_merge(w));
        HIP_TRY(launch_flip(w, k));
    }
    if (measure) HIP_TRY(launch_measure(w, n_sweeps - 1));
    if (measure || dev_status)
        HIP_TRY(launch_emit_row(ring, STATIC_SLOTS, first_sweep + n_sweeps - 1, g.q, g.N,
                                measure ? dev_obs + (size_t)(n_sweeps - 1) * W : nullptr, &st->err, dev_status, stream));
    return SW_OK;
}
