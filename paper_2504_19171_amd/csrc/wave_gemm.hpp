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
//   A(i, k) = ta ? a[k + i*lda] : a[i + k*lda]     i < 32 (rows >= avalid read as 0)
//   B(k, j) = tb ? b[j + k*ldb] : b[k + j*ldb]     j < 32
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

// Per-wavefront LDS staging: each wavefront fetches 16-deep chunks of its own
// A (32 x 16) and B (16 x 32) with loads that run along the contiguous
// dimension of each operand (coalesced whatever the orientation), writes them
// to its private LDS area as [k][i] / [k][j], and feeds the MFMAs from there.
#define WS_LD 33
#define WS_WAVE_DOUBLES (2 * 16 * WS_LD)
#define WS_SMEM_DOUBLES (4 * WS_WAVE_DOUBLES)

// Order the LDS accesses of one wavefront (its lanes run in lockstep; this
// waits for outstanding LDS operations and stops compiler reordering).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 8 doubles of a 16-deep chunk of operand (x = output index, k = reduction).
//   contig_x: element (x, k) at p[x + k*ld], else at p[k + x*ld].
__device__ inline void ws_fetch(const double* p, int64_t ld, int contig_x, int valid, int k0, int coh,
                                double r[8]) {
    // offsets stay inside one operand tile (< 2^31 doubles)
    const double* b = uniform_ptr(p);
    const int l = threadIdx.x & 63;
    const int ldi = (int)ld;
    int o, st;
    bool ok[8];
    if (contig_x) {
        const int x = l & 31;
        o = x + (k0 + (l >> 5)) * ldi;
        st = 2 * ldi;
#pragma unroll
        for (int q = 0; q < 8; ++q) ok[q] = x < valid;
    } else {
        const int x0 = l >> 4;
        o = (k0 + (l & 15)) + x0 * ldi;
        st = 4 * ldi;
#pragma unroll
        for (int q = 0; q < 8; ++q) ok[q] = x0 + 4 * q < valid;
    }
    if (coh) {
#pragma unroll
        for (int q = 0; q < 8; ++q) r[q] = ok[q] ? ld_coh(b + o + q * st) : 0.0;
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) r[q] = ok[q] ? b[o + q * st] : 0.0;
    }
}

__device__ inline void ws_stash(double* s, int contig_x, const double r[8]) {
    const int l = threadIdx.x & 63;
    if (contig_x) {
#pragma unroll
        for (int q = 0; q < 8; ++q) s[((l >> 5) + 2 * q) * WS_LD + (l & 31)] = r[q];
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) s[(l & 15) * WS_LD + (l >> 4) + 4 * q] = r[q];
    }
}

#define WS_PD 2   // default number of 16-deep chunks in flight per wavefront (registers)

__device__ inline void ws_mma16(dbl4 (&acc)[2][2], const double* sA, const double* sB) {
    const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
        const double* pa = sA + (kk + lk) * WS_LD + li;
        const double* pb = sB + (kk + lk) * WS_LD + li;
        const double a0 = pa[0], a1 = pa[16], b0 = pb[0], b1 = pb[16];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

// acc += A(:, k0:k1) * B(k0:k1, :) for this wavefront; k0, k1 multiples of 16.
// sw: this wavefront's LDS area (WS_WAVE_DOUBLES doubles).  Up to PD
// chunks are being fetched while one is multiplied.
template <int PD = WS_PD>
__device__ inline void wave_seg(dbl4 (&acc)[2][2], const Seg& sg, int k0, int k1, double* sw) {
    const int nch = (k1 - k0) >> 4;
    if (nch <= 0) return;
    const int ca = !sg.ta, cb = sg.tb;   // A normal / B transposed: contiguous along x
    double* sA = sw;
    double* sB = sw + 16 * WS_LD;
    double ra[PD][8], rb[PD][8];
#pragma unroll
    for (int p = 0; p < PD; ++p) {
        if (p < nch) {
            ws_fetch(sg.a, sg.lda, ca, sg.avalid, k0 + 16 * p, sg.ca, ra[p]);
            ws_fetch(sg.b, sg.ldb, cb, 32, k0 + 16 * p, sg.cb, rb[p]);
        }
    }
    int it = 0;
    for (; it + PD <= nch; it += PD) {
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            wave_lds_sync();
            ws_stash(sA, ca, ra[p]);
            ws_stash(sB, cb, rb[p]);
            wave_lds_sync();
            const int nx = it + p + PD;
            if (nx < nch) {
                ws_fetch(sg.a, sg.lda, ca, sg.avalid, k0 + 16 * nx, sg.ca, ra[p]);
                ws_fetch(sg.b, sg.ldb, cb, 32, k0 + 16 * nx, sg.cb, rb[p]);
            }
            ws_mma16(acc, sA, sB);
        }
    }
#pragma unroll
    for (int p = 0; p < PD; ++p) {
        if (it + p < nch) {
            wave_lds_sync();
            ws_stash(sA, ca, ra[p]);
            ws_stash(sB, cb, rb[p]);
            wave_lds_sync();
            ws_mma16(acc, sA, sB);
        }
    }
    wave_lds_sync();
}

// Run this wavefront's share of a reduction made of nseg segments of total
// length ktot (a multiple of 16); seg(q) returns segment q.  The reduction is
// cut at multiples of 16 into four consecutive pieces, one per wavefront.
// smem: WS_SMEM_DOUBLES doubles.
// Only the range [kbeg, kend) of the reduction is done when kend >= 0
// (multiples of 16).
template <int PD = WS_PD, class F>
__device__ inline void wave_segs(dbl4 (&acc)[2][2], int nseg, int ktot, double* smem, F&& seg, int kbeg = 0,
                                 int kend = -1) {
    if (kend < 0) kend = ktot;
    const int chunks = (kend - kbeg) >> 4;
    const int per = (chunks + 3) >> 2;
    const int w = threadIdx.x >> 6;
    int kb = kbeg + 16 * per * w, ke = kbeg + 16 * per * (w + 1);
    if (ke > kend) ke = kend;
    if (kb > kend) kb = kend;
    double* sw = smem + w * WS_WAVE_DOUBLES;
    int s0 = 0;
    for (int q = 0; q < nseg && s0 < ke; ++q) {
        const Seg sg = seg(q);
        const int lo = kb > s0 ? kb : s0;
        const int hi = ke < s0 + sg.K ? ke : s0 + sg.K;
        if (lo < hi) wave_seg<PD>(acc, sg, lo - s0, hi - s0, sw);
        s0 += sg.K;
    }
}

#define WR_LD 33
#define WR_SMEM_DOUBLES (4 * 32 * WR_LD)

// Sum the four wavefronts' accumulators (wave 0 + 1 + 2 + 3, in that order)
// into red[j*WR_LD + i] (column-major 32 x 32).  smem may be the staging area
// of wave_segs (WS_SMEM_DOUBLES >= WR_SMEM_DOUBLES).  Ends with a barrier.
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
