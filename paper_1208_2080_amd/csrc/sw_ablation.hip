// The paper's own labelling scheme, kept only as a measured comparison for the
// tile union-find of the sweep (no sweep uses it): Kalentev-style iterated
// label equivalence (Sec. 2, last paragraphs).  Every site starts as its own
// label; a scan kernel compares each site's label with the labels of its
// bonded neighbours and lowers the entry indexed by its label to the smallest
// of them; an analysis kernel walks every site's label chain to its end; the
// host repeats both until a scan changes nothing.  The result is the smallest
// site index of every cluster, as the sweep's labeller gives.
#include <hip/hip_runtime.h>

#include "sw_device.hpp"
#include "sw_kernels.hpp"

namespace swmi {

namespace {

// Bond of site (x, y) in plane p (0: +x, 1: +y) from the sweep's tile-major
// bond words (tiles of 64 columns by 2^log2ty rows).
__device__ __forceinline__ bool bond_at(const LatDesc& d, uint32_t log2ty, uint32_t x, uint32_t y, uint32_t p)
{
    const uint32_t tyi = y >> log2ty, r = y & ((1u << log2ty) - 1u);
    const size_t tile = (size_t)tyi * d.ntx + (x >> 6);
    const uint64_t w = glb(d.bonds)[((tile * 2 + p) << log2ty) + r];
    return (w >> (x & 63u)) & 1u;
}

__global__ __launch_bounds__(256) void k_le_init(const LatDesc* descs, uint32_t* lab)
{
    const LatDesc d = descs[0];
    const uint32_t x = blockIdx.x * 64 + (threadIdx.x & 63u), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= d.L || y >= d.L) return;
    const uint32_t i = y * d.L + x;   // site indices fit 32 bits (N <= 2^32)
    glb(lab)[i] = i;
}

// Scan: the smallest label among the site and its bonded neighbours lowers
// the entry indexed by the site's own label.
__global__ __launch_bounds__(256) void k_le_scan(const LatDesc* descs, uint32_t log2ty, uint32_t* lab, uint32_t* flag)
{
    const LatDesc d = descs[0];
    const uint32_t L = d.L;
    const uint32_t x = blockIdx.x * 64 + (threadIdx.x & 63u), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    bool changed = false;
    if (x < L && y < L) {
        const gptr<uint32_t> g = glb(lab);
        const uint32_t xl = x ? x - 1 : L - 1, xr = (x + 1 == L) ? 0 : x + 1;
        const uint32_t yu = y ? y - 1 : L - 1, yd = (y + 1 == L) ? 0 : y + 1;
        const uint32_t l = g[(size_t)y * L + x];
        uint32_t m = l;
        if (bond_at(d, log2ty, x, y, 0)) m = min(m, g[(size_t)y * L + xr]);
        if (bond_at(d, log2ty, xl, y, 0)) m = min(m, g[(size_t)y * L + xl]);
        if (bond_at(d, log2ty, x, y, 1)) m = min(m, g[(size_t)yd * L + x]);
        if (bond_at(d, log2ty, x, yu, 1)) m = min(m, g[(size_t)yu * L + x]);
        if (m < l) {
            // the atomic only when it can lower the entry: a giant cluster's
            // sites all target one entry, and most of them find it lowered already
            if (m < g[l]) min_coherent(g + l, m);
            changed = true;
        }
    }
    if (__builtin_amdgcn_ballot_w64(changed) && (threadIdx.x & 63u) == 0)
        __hip_atomic_store(glb(flag), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Analysis: every site follows its label chain (strictly decreasing indices)
// to the end and keeps that label.
__global__ __launch_bounds__(256) void k_le_analysis(const LatDesc* descs, uint32_t* lab)
{
    const LatDesc d = descs[0];
    const uint32_t x = blockIdx.x * 64 + (threadIdx.x & 63u), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= d.L || y >= d.L) return;
    const gptr<uint32_t> g = glb(lab);
    const size_t i = (size_t)y * d.L + x;
    uint32_t l = g[i], p = g[l];
    while (p < l) {
        l = p;
        p = g[l];
    }
    if (p != l) __hip_atomic_fetch_or(glb(d.err), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    g[i] = l;
}

dim3 le_grid(uint32_t L) { return dim3((L + 63) / 64, (L + 3) / 4); }

}  // namespace

hipError_t launch_le_init(const LatDesc* descs, uint32_t L, uint32_t* lab, hipStream_t s)
{
    hipLaunchKernelGGL(k_le_init, le_grid(L), dim3(256), 0, s, descs, lab);
    return hipGetLastError();
}

hipError_t launch_le_iteration(const LatDesc* descs, uint32_t L, uint32_t ty, uint32_t* lab, uint32_t* flag,
                               hipStream_t s)
{
    uint32_t log2ty = 0;
    while ((1u << log2ty) < ty) ++log2ty;
    if ((1u << log2ty) != ty) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_le_scan, le_grid(L), dim3(256), 0, s, descs, log2ty, lab, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_le_analysis, le_grid(L), dim3(256), 0, s, descs, lab);
    return hipGetLastError();
}

}  // namespace swmi
