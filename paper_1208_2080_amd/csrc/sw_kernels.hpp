// Host-side launchers of the SW kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sw_layout.hpp"

namespace swmi {

// What one sweep phase runs over: the tiles of descs[0] when map is null
// (nitems = its tile count), else the work items of map (batched form).
struct Work {
    const LatDesc* descs;
    const WorkItem* map;
    uint32_t nitems;
    uint32_t ty;
    hipStream_t stream;
    bool cluster = false;  // some lattice measures cluster-size sums
    bool xy = false;       // XY lattices (Wolff's embedded clusters)
};

hipError_t launch_bond_label(const Work& w, uint32_t k, uint32_t flags);
hipError_t launch_merge(const Work& w);
hipError_t launch_flip(const Work& w, uint32_t k);
hipError_t launch_measure(const Work& w, uint32_t k);
// cluster-size sums of the sweep counter + k (after its flip), for the
// lattices that measure them
hipError_t launch_cluster_sums(const Work& w, uint32_t k);
// measurement after n_each[lattice] sweeps of each lattice (batched form)
hipError_t launch_measure_each(const Work& w, const uint32_t* n_each);
hipError_t launch_init(const LatDesc* descs, uint32_t lat, size_t N, uint32_t random_start, hipStream_t s);

// XY lattices: the bond step of sweep counter + k (flags bit 0: also measure
// the incoming configuration; bit 1: only measure the current one, k =
// 0xFFFFFFFF naming the last sweep), the labeller over those bonds, the flip
// as reflections, and the initial angles.
hipError_t launch_xy_bonds(const Work& w, uint32_t k, uint32_t flags);
hipError_t launch_label_preset(const Work& w);
hipError_t launch_flip_xy(const Work& w, uint32_t k);
hipError_t launch_xy_init(const LatDesc* descs, size_t N, uint32_t random_start, hipStream_t s);
// Lattices of L <= WHOLE_LMAX swept whole in one workgroup each (descs[list[b]]
// for workgroup b, or descs[b] without a list), n_each[lattice] (or n_uniform)
// sweeps each from sweep counter + k0; lmax: the largest L among them.  flags
// bit 0: also write the last sweep's labels (smallest site indices) and bond
// words (tile-major, ty rows per tile); bit 1: leave the sweep counters (else
// set past the last sweep).
hipError_t launch_whole(const LatDesc* descs, const uint32_t* list, uint32_t count, uint32_t lmax, uint32_t k0,
                        uint32_t n_uniform, const uint32_t* n_each, uint32_t flags, uint32_t ty, hipStream_t s);
// Labels of rows [ya, yb) of the last sweep resolved to smallest site
// indices, written from the base of the label region ((yb - ya) L <= N / 2).
hipError_t launch_resolve(const LatDesc* descs, uint32_t lat, uint32_t ntiles, uint32_t ty, uint32_t ya, uint32_t yb,
                          hipStream_t s);
// Sum the NCOPY partial copies of n ring records of `words` words (copies
// `stride` words apart), from slot slot0 on (wrapping at `slots`), into
// out[n][words].
hipError_t launch_ring_sum(const int64_t* ring, int64_t* out, uint32_t slots, uint32_t slot0, uint32_t n,
                           uint32_t words, uint32_t stride, hipStream_t s);
hipError_t launch_bump(const LatDesc* descs, uint32_t count, const uint32_t* n_each, uint32_t n, hipStream_t s);

// No-allocation entry point: copy the descriptor d to d_out, clear the error
// flag, set the sweep counter and zero ring_words words of the ring (all in
// caller-independent scratch).
hipError_t launch_static_setup(const LatDesc& d, LatDesc* d_out, DevState* st, uint32_t counter, int64_t* ring,
                               uint32_t ring_words, hipStream_t s);
// Ring record `slot` (of `slots`) of a lattice with q states and N sites as one
// observable row [n_unsat, n_active, n_0..n_{q-1}] at row (if row is not null);
// *err copied to *status (if status is not null).
hipError_t launch_emit_row(const int64_t* ring, uint32_t slots, uint32_t slot, uint32_t q, uint64_t N, int64_t* row,
                           const uint32_t* err, uint32_t* status, hipStream_t s);

// Iterated label equivalence over the bonds of descs[0]'s last sweep (a
// comparison for the tile labeller; sw_ablation.hip): lab[i] = i, then one
// scan + analysis pass per call of launch_le_iteration, which sets *flag when
// the scan lowered a label.
hipError_t launch_le_init(const LatDesc* descs, uint32_t L, uint32_t* lab, hipStream_t s);
hipError_t launch_le_iteration(const LatDesc* descs, uint32_t L, uint32_t ty, uint32_t* lab, uint32_t* flag,
                               hipStream_t s);

}  // namespace swmi
