// device.hpp -- small device helpers shared by the HIP kernels of libsmi.
#pragma once

#include <hip/hip_runtime.h>

namespace smi {

// first z of the 32-float-aligned (128-byte) storage line that contains node z, with the
// ghost frame of 8 nodes in front of node 0
__host__ __device__ __forceinline__ int zalign(int z) { return ((z + 8) & ~31) - 8; }

// Compact index of node i inside the CPML slabs of an axis with M nodes: [0, nb) and
// [M - nb - 1, M) map to [0, 2 nb + 1); interior nodes return -1.
__device__ __forceinline__ int slab_index(int i, int M, int nb) {
    return i < nb ? i : (i >= M - nb - 1 ? i - (M - nb - 1) + nb : -1);
}

// f[k + off*stride] if the shifted index stays inside [0, M), else 0 (the padded grid is
// surrounded by zeros).  The address is clamped so that no lane ever reads out of bounds.
__device__ __forceinline__ float ldz(const float *__restrict__ f, long long k, int i, int off,
                                     long long stride, int M) {
    bool ok = (unsigned)(i + off) < (unsigned)M;
    float v = f[k + (ok ? (long long)off * stride : 0)];
    return ok ? v : 0.f;
}

// The amplitude a source adds to p at one node, rounded once: contraction is off here, so the
// product never fuses with the add or subtract that uses it (a plain product, or __fmul_rn,
// which HIP defines as one, would become an FMA there).  The forward injection adds this value
// and the reconstruction subtracts the same value, so a node that held zero before the
// injection returns to exactly zero.
__device__ __forceinline__ float src_amp(float scale, float stf) {
#pragma clang fp contract(off)
    return scale * stf;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Give each
// XCD a contiguous range of logical work items so that neighbouring tiles, which share halos
// and model data, are resident in the same L2.
__device__ __forceinline__ int xcd_remap(int wg, int G) {
    int xcd = wg & 7, slot = wg >> 3;
    int per = G >> 3, rem = G & 7;
    return xcd * per + min(xcd, rem) + slot;
}

}  // namespace smi
