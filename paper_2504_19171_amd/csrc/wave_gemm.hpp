// 32 x 32 output block of an FP64 product on one workgroup of 4 wavefronts,
// the reduction dimension split four ways (one piece per wavefront) and the
// four partial blocks summed through LDS in a fixed order, so results do not
// depend on timing.  Used where latency matters more than throughput: a
// small output block spread over a whole workgroup.
//
// v_mfma_f64_16x16x4_f64 lane layout (lane l): A[l%16][l/16], B[l/16][l%16],
// D element r = D[4r + l/16][l%16].
#pragma once
#include "common.hpp"

// One contiguous piece of the reduction dimension.
//   A(i, k) = ta ? a[k + i*lda] : a[i + k*lda]     i < 32
//   B(k, j) = tb ? b[j + k*ldb] : b[k + j*ldb]     j < 32
//   avalid: rows of A that exist (even, and 32 when ta == 1).  Rows past it
//     are filled with copies of existing rows, so the output rows >= avalid
//     are meaningless and the caller discards them.
//   ca / cb: read A / B with device-coherent loads (data written by other
//   workgroups of the same kernel)
struct Seg {
    const double* a;
    const double* b;
    int64_t lda, ldb;
    int ta, tb;
    int K;        // multiple of 16
    int avalid;
    int ca, cb;
};

__device__ inline Seg mkseg(const double* a, int64_t lda, int ta, const double* b, int64_t ldb, int tb, int K,
                            int avalid = 32, int ca = 0, int cb = 0) {
    Seg s;
    s.a = a; s.b = b; s.lda = lda; s.ldb = ldb; s.ta = ta; s.tb = tb; s.K = K; s.avalid = avalid;
    s.ca = ca; s.cb = cb;
    return s;
}

// Per-wavefront LDS staging with direct loads: a KC-deep chunk of A (32 x KC)
// and of B (KC x 32), KC = 16 or 8, goes from memory straight into the
// wavefront's private LDS area (global_load_lds_dwordx4: lane l's 16 bytes
// land at 16*l from the instruction's base, 1 KB per instruction, KC/4
// instructions per operand), two chunks in flight in two buffers.  No
// registers hold data in flight and nothing is copied into LDS by the
// wavefront itself.  Each lane fetches two consecutive doubles along the
// contiguous dimension of its operand:
//   contiguous along x (A with ta == 0, B with tb == 1): element (x, k) at
//     [k*32 + x];
//   contiguous along k: element (x, k) at [x*KC + 2*((k/2) ^ s(x)) + k%2],
//     s(x) = x%8 (KC = 16) or (x/4)%4 (KC = 8): the pairs of a row permuted by
//     the row index, so that the 16 rows a matrix-core operand read touches
//     fall in different LDS banks.
// Sixteen-deep chunks keep fewer waits per product; eight-deep ones halve the
// LDS area, so that three workgroups fit on one compute unit.
template <int KC>
struct WS {
    static constexpr int CHUNK = 2 * 32 * KC;     // A then B
    static constexpr int WAVE = 2 * CHUNK;        // two buffers
    static constexpr int SMEM = 4 * WAVE;         // four wavefronts
    static constexpr int VMCNT_CHUNK = KC == 16 ? 0x0F78 : 0x0F74;   // s_waitcnt vmcnt(KC/2)
};

typedef __attribute__((address_space(3))) void lds_void_t;

// Issue the loads of one 32 x KC operand chunk (x = output index, k =
// reduction index, k0 its first k) into dst (32 KC doubles of LDS).
//   contig_x: element (x, k) at p[x + k*ld], else at p[k + x*ld].
// COH: device-coherent loads.  Offsets stay inside one operand tile.
template <int KC, int COH>
__device__ inline void wl_fetch(const double* p, int64_t ld, int contig_x, int valid, int k0, double* dst) {
    const double* b = uniform_ptr(p);
    const int l = threadIdx.x & 63;
    const int ldi = (int)ld;
    if (contig_x) {
        // instruction q: k = k0 + 4q + l/16, rows 2*(l%16), +1 (a pair past
        // `valid` reads the last existing pair)
        const int x2 = imin_(2 * (l & 15), valid - 2);
        const double* g = b + x2 + (int64_t)(k0 + (l >> 4)) * ldi;
#pragma unroll
        for (int q = 0; q < KC / 4; ++q)
            __builtin_amdgcn_global_load_lds((const void*)(g + (int64_t)(4 * q) * ldi),
                                             (lds_void_t*)(dst + 128 * q), 16, 0, COH ? 16 : 0);
    } else if (KC == 16) {
        // instruction q: row x = 8q + l/8, pair c = (l%8) ^ (x%8) of k
        const int xl = l >> 3, c = (l & 7) ^ xl;
        const double* g = b + (k0 + 2 * c) + (int64_t)xl * ldi;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            __builtin_amdgcn_global_load_lds((const void*)(g + (int64_t)(8 * q) * ldi),
                                             (lds_void_t*)(dst + 128 * q), 16, 0, COH ? 16 : 0);
    } else {
        // instruction q: row x = 16q + l/4, pair c = (l%4) ^ ((x/4)%4) of k
        const int c = (l & 3) ^ ((l >> 4) & 3);
        const double* g = b + (k0 + 2 * c) + (int64_t)(l >> 2) * ldi;
#pragma unroll
        for (int q = 0; q < 2; ++q)
            __builtin_amdgcn_global_load_lds((const void*)(g + (int64_t)(16 * q) * ldi),
                                             (lds_void_t*)(dst + 128 * q), 16, 0, COH ? 16 : 0);
    }
}

// LDS index of element (x, k) of a chunk (see above).
template <int KC>
__device__ inline int wl_at(int contig_x, int x, int k) {
    if (contig_x) return k * 32 + x;
    return KC == 16 ? x * 16 + 2 * ((k >> 1) ^ (x & 7)) + (k & 1) : x * 8 + 2 * ((k >> 1) ^ ((x >> 2) & 3)) + (k & 1);
}

// LDS byte address of a pointer into LDS.
__device__ inline uint32_t lds_addr(const double* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) double*)p;
}

// Four LDS reads and the wait for them in one block.  The compiler knows the
// direct loads write LDS but cannot tell which buffer, so before any LDS read
// it can see it would wait for every load in flight, the next chunk's too;
// reads it cannot see leave the waits to wave_seg_t, which knows the order.
__device__ inline void wl_read4(uint32_t pa0, uint32_t pa1, uint32_t pb0, uint32_t pb1, double& a0, double& a1,
                                double& b0, double& b1) {
    asm volatile(
        "ds_read_b64 %0, %4\n\t"
        "ds_read_b64 %1, %5\n\t"
        "ds_read_b64 %2, %6\n\t"
        "ds_read_b64 %3, %7\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(a0), "=&v"(a1), "=&v"(b0), "=&v"(b1)
        : "v"(pa0), "v"(pa1), "v"(pb0), "v"(pb1)
        : "memory");
}

// acc += the chunk in buf (A at buf, B at buf + 32 KC).
template <int KC>
__device__ inline void wl_mma(dbl4 (&acc)[2][2], const double* buf, int ca, int cb) {
    const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const uint32_t sa = lds_addr(buf), sb = lds_addr(buf + 32 * KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
        const int k = kk + lk;
        double a0, a1, b0, b1;
        wl_read4(sa + 8u * wl_at<KC>(ca, li, k), sa + 8u * wl_at<KC>(ca, li + 16, k), sb + 8u * wl_at<KC>(cb, li, k),
                 sb + 8u * wl_at<KC>(cb, li + 16, k), a0, a1, b0, b1);
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

// s_waitcnt immediates, gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8; a counter at its maximum is not waited for.
//   vmcnt(0) (expcnt 7, lgkmcnt 15); lgkmcnt(0) (vmcnt 63, expcnt 7)
#define WL_VMCNT0 0x0F70
#define WL_LGKM0 0xC07F

template <int KC, int CA, int CB>
__device__ inline void wl_issue(const Seg& sg, int ca, int cb, int avalid, int k, double* buf) {
    wl_fetch<KC, CA>(sg.a, sg.lda, ca, avalid, k, buf);
    wl_fetch<KC, CB>(sg.b, sg.ldb, cb, 32, k, buf + 32 * KC);
}

// acc += A(:, k0:k1) * B(k0:k1, :) for this wavefront; k0, k1 multiples of KC.
// sw: this wavefront's LDS area (WS<KC>::WAVE doubles), which holds nothing
// else while this runs.  Chunk c+2 is fetched into the buffer of chunk c
// once the products of chunk c have read it.  The vmcnt waits assume no other
// memory access of this wavefront is issued in between (loads issued before
// are older and complete first).
template <int KC, int CA, int CB>
__device__ inline void wave_seg_t(dbl4 (&acc)[2][2], const Seg& sg, int k0, int k1, double* sw) {
    const int nch = __builtin_amdgcn_readfirstlane((k1 - k0) / KC);
    if (nch <= 0) return;
    const int ca = __builtin_amdgcn_readfirstlane(!sg.ta), cb = __builtin_amdgcn_readfirstlane(sg.tb);
    const int avalid = __builtin_amdgcn_readfirstlane(sg.avalid);
    // the previous user of this LDS area has read it
    __builtin_amdgcn_s_waitcnt(WL_LGKM0);
    __builtin_amdgcn_wave_barrier();
    wl_issue<KC, CA, CB>(sg, ca, cb, avalid, k0, sw);
    if (nch > 1) wl_issue<KC, CA, CB>(sg, ca, cb, avalid, k0 + KC, sw + WS<KC>::CHUNK);
    for (int c = 0; c < nch; ++c) {
        double* buf = sw + (c & 1) * WS<KC>::CHUNK;
        // chunk c has landed in LDS (chunk c+1's KC/2 loads may still fly)
        if (c + 1 < nch) __builtin_amdgcn_s_waitcnt(WS<KC>::VMCNT_CHUNK);
        else __builtin_amdgcn_s_waitcnt(WL_VMCNT0);
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
        wl_mma<KC>(acc, buf, ca, cb);
        if (c + 2 < nch) {
            // every read of this buffer has returned before it is refilled
            __builtin_amdgcn_s_waitcnt(WL_LGKM0);
            __builtin_amdgcn_wave_barrier();
            asm volatile("" ::: "memory");
            wl_issue<KC, CA, CB>(sg, ca, cb, avalid, k0 + KC * (c + 2), buf);
        }
    }
    __builtin_amdgcn_s_waitcnt(WL_LGKM0);
    __builtin_amdgcn_wave_barrier();
}

template <int KC>
__device__ inline void wave_seg(dbl4 (&acc)[2][2], const Seg& sg, int k0, int k1, double* sw) {
    const int c = __builtin_amdgcn_readfirstlane((sg.ca ? 1 : 0) | (sg.cb ? 2 : 0));
    if (c == 1) wave_seg_t<KC, 1, 0>(acc, sg, k0, k1, sw);
    else if (c == 2) wave_seg_t<KC, 0, 1>(acc, sg, k0, k1, sw);
    else if (c == 3) wave_seg_t<KC, 1, 1>(acc, sg, k0, k1, sw);
    else wave_seg_t<KC, 0, 0>(acc, sg, k0, k1, sw);
}

// Run this wavefront's share of a reduction made of nseg segments of total
// length ktot (a multiple of 16); seg(q) returns segment q.  The reduction is
// cut at multiples of 16 into four consecutive pieces, one per wavefront.
// smem: WS<KC>::SMEM doubles.
// Only the range [kbeg, kend) of the reduction is done when kend >= 0
// (multiples of 16).
template <int KC, class F>
__device__ inline void wave_segs(dbl4 (&acc)[2][2], int nseg, int ktot, double* smem, F&& seg, int kbeg = 0,
                                 int kend = -1) {
    if (kend < 0) kend = ktot;
    const int chunks = (kend - kbeg) >> 4;
    const int per = (chunks + 3) >> 2;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int kb = kbeg + 16 * per * w, ke = kbeg + 16 * per * (w + 1);
    if (ke > kend) ke = kend;
    if (kb > kend) kb = kend;
    double* sw = smem + w * WS<KC>::WAVE;
    int s0 = 0;
    for (int q = 0; q < nseg && s0 < ke; ++q) {
        const Seg sg = seg(q);
        const int lo = kb > s0 ? kb : s0;
        const int hi = ke < s0 + sg.K ? ke : s0 + sg.K;
        if (lo < hi) wave_seg<KC>(acc, sg, lo - s0, hi - s0, sw);
        s0 += sg.K;
    }
}

#define WR_LD 33
#define WR_SMEM_DOUBLES (4 * 32 * WR_LD)

// Sum the four wavefronts' accumulators (wave 0 + 1 + 2 + 3, in that order)
// into red[j*WR_LD + i] (column-major 32 x 32).  smem (WR_SMEM_DOUBLES
// doubles, which may be the staging area of wave_segs) must not overlap red.
// Ends with a barrier.
__device__ inline void wave_reduce(const dbl4 (&acc)[2][2], double* smem, double* red) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    double* mine = smem + w * 32 * WR_LD;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                mine[(tj * 16 + (l & 15)) * WR_LD + ti * 16 + 4 * r + (l >> 4)] = acc[ti][tj][r];
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int i = e & 31, j = e >> 5;
        const int o = j * WR_LD + i;
        double v = smem[o];
        v += smem[32 * WR_LD + o];
        v += smem[64 * WR_LD + o];
        v += smem[96 * WR_LD + o];
        red[o] = v;
    }
    __syncthreads();
}
