// Shared definitions of the HIP path: tile layout and small helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Device-side view of the tile layout (see include/stiles.h for the format).
struct Lay {
    int64_t nb;        // order of the band part
    int64_t w;         // half-bandwidth, clamped to nb-1
    int64_t nt;        // N: band tile columns
    int64_t off_band, off_arrow, off_corner, total;
    int b;             // tile size
    int bt;            // B: tile half-bandwidth
    int ap;            // arrow rows rounded up to 16 (0 when there is no arrow)
    int a;             // arrow rows
    int p2s;           // parts of each Phase 2 output's sum: 3, or 2 (k = J+2 joins the far part)

    // Offset (in doubles) of band tile (J+d, J).
    __host__ __device__ int64_t band(int64_t J, int d) const {
        return off_band + (J * (int64_t)(bt + 1) + d) * (int64_t)b * b;
    }
    // Offset of arrow tile J (rows nb.., tile column J), a_p x b.
    __host__ __device__ int64_t arrow(int64_t J) const { return off_arrow + J * (int64_t)ap * b; }
    __host__ __device__ int64_t corner() const { return off_corner; }
    // Number of band tiles below the diagonal in tile column J.
    __host__ __device__ int s(int64_t J) const {
        int64_t r = nt - 1 - J;
        return (int)(r < bt ? r : bt);
    }
};

// Row blocks of 64 rows in an arrow tile (a_p rows, last block may be partial).
__host__ __device__ inline int arrow_blocks(int ap) { return (ap + 63) / 64; }
__host__ __device__ inline int imin_(int x, int y) { return x < y ? x : y; }
__host__ __device__ inline int imax_(int x, int y) { return x > y ? x : y; }
__host__ __device__ inline int64_t imax64(int64_t x, int64_t y) { return x > y ? x : y; }

// The workgroups of a launch are dealt to the 8 XCDs in turn (workgroup i to
// XCD i mod 8), and each XCD has its own L2.  xcd_block renumbers them so that
// every XCD holds one contiguous run of logical blocks: neighbouring blocks,
// which read the same operand strips, then share one L2 instead of fetching
// the strip once per XCD.  A bijection on [0, G) for any G, so correctness
// does not depend on the dealing order.
__host__ __device__ inline int xcd_block(int b, int G) {
    const int x = b & 7, slot = b >> 3, q = G >> 3, r = G & 7;
    return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// Global (device) memory address space.  Every pointer the kernels read or
// write through is global memory, but a pointer the compiler cannot trace
// back to a kernel argument (one rebuilt from an integer, say) is generic,
// and a generic access becomes a FLAT instruction.  FLAT loads and stores
// count on the LDS counter as well as the memory one, so every wait for an
// LDS access would also wait for every memory access in flight, and loads
// issued ahead of their use would no longer overlap anything.  Casting to
// this address space keeps such accesses GLOBAL instructions.
#define GLOBAL_AS __attribute__((address_space(1)))

// The same pointer in every lane, held in scalar registers: lets loads use a
// scalar base plus a 32-bit per-lane offset instead of 64-bit addresses.
// The pointer is rebuilt in the global address space (then converted back),
// so accesses through it stay GLOBAL instructions.  p must point to device
// memory.
__device__ inline const double* uniform_ptr(const double* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const double*)(const GLOBAL_AS double*)(((uint64_t)hi << 32) | lo);
}

// base[idx] for a wave-uniform base and idx < 2^29: the byte offset is a
// 32-bit value, so the load can use the scalar-base + vector-offset form and
// needs no 64-bit address per lane.
__device__ inline double ld_s(const double* base, uint32_t idx) {
    uint32_t o = idx << 3;
    asm volatile("" : "+v"(o));   // keep the 64-bit address out of loop-invariant code motion
    return *(const GLOBAL_AS double*)((const char*)base + o);
}

__device__ inline void st_s(double* base, uint32_t idx, double v) {
    uint32_t o = idx << 3;
    asm volatile("" : "+v"(o));
    *(GLOBAL_AS double*)((char*)base + o) = v;
}

// base[idx] = v as a device-coherent store (see st_coh below), with the same
// scalar-base + 32-bit offset addressing as st_s.
__device__ inline void st_coh_s(double* base, uint32_t idx, double v) {
    uint32_t o = idx << 3;
    asm volatile("" : "+v"(o));
    __hip_atomic_store((GLOBAL_AS double*)((char*)base + o), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_coh_s(const double* base, uint32_t idx) {
    uint32_t o = idx << 3;
    asm volatile("" : "+v"(o));
    return __hip_atomic_load((const GLOBAL_AS double*)((const char*)base + o), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Device-coherent load / store of one double (agent-scope relaxed atomics:
// they bypass the non-coherent cache levels, see persist.hpp).
__device__ inline double ld_coh(const double* p) {
    return __hip_atomic_load((const GLOBAL_AS double*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_coh(double* p, double v) {
    __hip_atomic_store((GLOBAL_AS double*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-coherent int load / fetch-and-add (counters and flags handed between
// workgroups), and the first error code of a kernel into *err (0 = none).
__device__ inline int ld_coh_i(const int* p) {
    return __hip_atomic_load((const GLOBAL_AS int*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int add_coh_i(int* p, int v) {
    return __hip_atomic_fetch_add((GLOBAL_AS int*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void set_error_once(int* err, int code) {
    int zero = 0;
    __hip_atomic_compare_exchange_strong((GLOBAL_AS int*)err, &zero, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
}
