// Cholesky of one diagonal tile (m <= 256, m a multiple of 64) by one
// workgroup of 1 + P3_PW wavefronts, left-looking over 16-column panels with a
// one-panel lookahead:
//   - wavefronts 1..P3_PW own the 16 x 16 row tiles I = w, w+P3_PW, ... of every
//     panel; the reduced current panel sits in LDS in transposed MFMA form
//     (lane (i, k) reads C[16I + i][c0 + 4r + k], the layout the matrix cores
//     take as the B operand, so the panel solve needs no shuffle);
//   - the diagonal 16 x 16 block is factored by wavefront 0 (one column per
//     lane, pivot columns broadcast along 16-lane rows with DPP, the inverse
//     formed in the same sweep; see p3_factor16), while the other wavefronts
//     reduce the panels ahead of it (see potrf3 below);
//   - the panel below is solved with the inverse of the diagonal block on the
//     matrix cores, L_Ip^T = Y_pp C_Ip^T.
// Also returns the inverses of the 16 x 16 diagonal blocks of L (for the
// panel TRSM below the tile) and the Neumaier pair of sum 2 log L_jj, and
// announces every finished panel to a concurrent consumer (see potrf3).
#pragma once
#include "common.hpp"
#include "tile_ops.hpp"

#define P3_LD 17
#define P3_PW 3                                    // panel wavefronts (1 .. P3_PW); wavefront 0 runs the diagonal chain
#define P3_NT (64 * (1 + P3_PW))                   // threads of a workgroup running potrf3
#define P3_SLOTS ((15 + P3_PW - 1) / P3_PW)        // row tiles I >= 1 per panel wavefront
#define P3_POOL 65       // 16 x 16 tiles of L alive at once at m = 256 (checked by p3_make_slots)
#define P3_POOL_128 17   // the same for m <= 128

// NPOOL: pool slots, P3_POOL for any m, P3_POOL_128 for m <= 128 (a smaller
// footprint lets more workgroups share a compute unit).
template <int NPOOL>
struct P3SmemT {
    double D[16 * P3_LD];          // diagonal block of the current panel, D(i, j) at D[j * P3_LD + i]
                                   // (both triangles on input to p3_factor16, L_pp in the lower one after)
    double Y[2][16 * P3_LD];       // Y_p = L_pp^{-1} in Y[p & 1], Y(i, j) at [i * P3_LD + j]: the panel
                                   // wavefronts still read Y_p while wavefront 0 forms Y_{p+1}
    double Dn[2][16 * P3_LD];      // next diagonal blocks (by parity), reduced up to two panels back
    double pool[NPOOL][256];       // tiles (I, k) of L in slots given by p3_slot: first the reduced tile in
                                   // transposed MFMA form (r * 64 + lane), then, solved in place,
                                   // L[16I + i][16k + j] at [j * 16 + i]
    double dg[256];                // diagonal of L, then 2 log L_jj
    double ps[64], pc[64];         // log det partial sums
    double lsum, lcomp;
    int fail;
};
using P3Smem = P3SmemT<P3_POOL>;

// sqrt(x) and 1/sqrt(x) from the hardware reciprocal square root and two
// Goldschmidt steps (a few ulp; the pivot decides nothing else).
__device__ inline void p3_sqrt_rsqrt(double x, double& s, double& r) {
    const double r0 = __builtin_amdgcn_rsq(x);
    double g = x * r0, h = 0.5 * r0;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    s = g;
    r = 2.0 * h;
}

// Workgroup barriers: LDS traffic only (the phases exchange data through LDS
// alone), or also every global access of every wavefront (before a panel is
// announced).  The "memory" clobber keeps the compiler from moving accesses
// across them.
__device__ inline void p3_bar_lds() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
__device__ inline void p3_bar_all() { asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ inline void p3_wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of lane K of this lane's 16-lane row (DPP row_newbcast:K).
template <int K>
__device__ __forceinline__ double p3_rowbcast(double v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xF, 0xF, true);
}
// The same for a lane index known at compile time after unrolling.
__device__ __forceinline__ double p3_rowbcast_i(double v, int i) {
    switch (i) {
    case 0: return p3_rowbcast<0>(v);
    case 1: return p3_rowbcast<1>(v);
    case 2: return p3_rowbcast<2>(v);
    case 3: return p3_rowbcast<3>(v);
    case 4: return p3_rowbcast<4>(v);
    case 5: return p3_rowbcast<5>(v);
    case 6: return p3_rowbcast<6>(v);
    case 7: return p3_rowbcast<7>(v);
    case 8: return p3_rowbcast<8>(v);
    case 9: return p3_rowbcast<9>(v);
    case 10: return p3_rowbcast<10>(v);
    case 11: return p3_rowbcast<11>(v);
    case 12: return p3_rowbcast<12>(v);
    case 13: return p3_rowbcast<13>(v);
    case 14: return p3_rowbcast<14>(v);
    default: return p3_rowbcast<15>(v);
    }
}

// Pivot K of the sweep in p3_factor16.  Lane j of every 16-lane row holds a
// column x of 16 values.  Before pivot K:
//   - a lane with j >= K holds column j of the partly reduced block A^(K)
//     (rows >= K; rows < K were cleared as they were used);
//   - a lane with j < K holds, in the rows whose role is the inverse (wrow),
//     Z = -d_j times column j of W^(K) = E_{K-1} ... E_0 (E_k: the k-th
//     elimination step, so W^(16) = U^{-1} for A = U diag(d) U^T, U unit lower
//     triangular), and in the other rows column j of U diag(d), kept.
// The step: d = A^(K)(K, K) from lane K; every lane forms q = x_K / d (for
// j > K the multiplier A^(K)(K, j) / d by symmetry; for j < K the entry
// W(K, j) scaled as above) and adds -A^(K)(i, K) q to its rows i > K, the
// pivot column A^(K)(i, K) coming from lane K.  Lane K itself changes no row
// below K: its column is U(:, K) d_K, which is also -d_K times column K of
// W^(K+1) below the diagonal, so only its diagonal entry becomes -d_K.
template <int K>
__device__ __forceinline__ void p3_pivot(double (&x)[16], double& dj, int& fail, int base, int j, bool wrow) {
    const double d = p3_rowbcast<K>(x[K]);
    double rr = __builtin_amdgcn_rcp(d);   // 1/d: hardware estimate and two Newton steps
    double e = fma(-d, rr, 1.0);
    rr = fma(rr, e, rr);
    e = fma(-d, rr, 1.0);
    rr = fma(rr, e, rr);
    if (!(d > 0.0) && fail < 0) fail = base + K;
    const double q = x[K] * rr;
    const double c = (j != K && (wrow || j > K)) ? q : 0.0;
    dj = (j == K) ? d : dj;
    x[K] = (j < K) ? x[K] : ((j == K) ? -x[K] : 0.0);
#pragma unroll
    for (int i = K + 1; i < 16; ++i) x[i] = fma(-p3_rowbcast<K>(x[i]), c, x[i]);
}
template <int K>
__device__ __forceinline__ void p3_pivots(double (&x)[16], double& dj, int& fail, int base, int j, bool wrow) {
    p3_pivot<K>(x, dj, fail, base, j, wrow);
    if constexpr (K < 15) p3_pivots<K + 1>(x, dj, fail, base, j, wrow);
}

// Factor the 16 x 16 block in sm.D (both triangles, symmetric) on one
// wavefront: L_pp into the lower part of sm.D ([col][row]; the upper part is
// overwritten with zeros), its diagonal into sm.dg, and Y = L_pp^{-1} into all
// of Y ([row][col], zeros above the diagonal).  A = U diag(d) U^T by the
// pivots of p3_pivot, each lane keeping one column, each pivot column
// broadcast along the lane rows (no LDS traffic inside the sweep); then
// L = U diag(d)^{1/2} and Y = diag(d)^{-1/2} U^{-1}, so
//   L(i, j) = [U diag(d)](i, j) / sqrt(d_j),   Y(i, j) = -Z(i, j) / (sqrt(d_i) d_j).
// Rows 0 and 2 of the wavefront carry the inverse, rows 1 and 3 the factor.
// *fail gets the first local column (base + j) whose pivot is not positive.
template <int NPOOL>
__device__ inline void p3_factor16(P3SmemT<NPOOL>& sm, double* Y, int base, int& fail) {
    const int lane = threadIdx.x & 63, j = lane & 15;
    const bool wrow = (lane & 16) == 0;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = sm.D[j * P3_LD + i];
    double dj = 1.0;
    p3_pivots<0>(x, dj, fail, base, j, wrow);
    double s, r;   // sqrt(d_j), 1/sqrt(d_j)
    p3_sqrt_rsqrt(dj, s, r);
    const double f = -(r * r);
    double g[16];   // -1/(sqrt(d_i) d_j)
#pragma unroll
    for (int i = 0; i < 16; ++i) g[i] = p3_rowbcast_i(r, i) * f;
    if (lane < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) Y[i * P3_LD + j] = x[i] * g[i];
    } else if (lane < 32) {
#pragma unroll
        for (int i = 0; i < 16; ++i) sm.D[j * P3_LD + i] = x[i] * r;
        sm.D[j * P3_LD + j] = s;
        sm.dg[base + j] = s;
    }
}

// Slots of the 16 x 16 tiles of L in the LDS pool, for np = 4, 8, 12, 16 row
// tiles.  Tile (I, k), I > k, enters the pool as a reduced tile of panel k
// during U(k-1) (the prologue for k = 0), is solved in place at S(k), and is
// read for the last time in U(I-2) (in U(I-1) when I = k+1; see potrf3).  A
// slot given back at the end of one U phase is handed out again from the next
// one on.  The table is packed one dword per lane for p3_slot: byte I/4 of
// lane 16 (I % 4) + k.
struct P3SlotPack {
    uint32_t w[4][64];
    int peak[4];
    int top[4];   // largest slot index handed out
};
constexpr P3SlotPack p3_make_slots() {
    P3SlotPack t{};
    for (int v = 0; v < 4; ++v) {
        const int np = 4 * (v + 1);
        int slot[16][16] = {};
        int fr[P3_POOL] = {};
        int nf = 0, live = 0, peak = 0;
        for (int q = P3_POOL - 1; q >= 0; --q) fr[nf++] = q;
        // an empty free list makes fr[-1] below, which stops the compilation
        int top = 0;
        for (int I = 1; I < np; ++I) { slot[I][0] = fr[--nf]; ++live; top = slot[I][0] > top ? slot[I][0] : top; }
        peak = live;
        for (int p = 0; p + 1 < np; ++p) {
            for (int I = p + 2; I < np; ++I) {
                slot[I][p + 1] = fr[--nf];
                ++live;
                top = slot[I][p + 1] > top ? slot[I][p + 1] : top;
            }
            if (live > peak) peak = live;
            if (p + 2 < np)
                for (int k = 0; k <= p; ++k) { fr[nf++] = slot[p + 2][k]; --live; }
            fr[nf++] = slot[p + 1][p];
            --live;
        }
        for (int I = 0; I < 16; ++I)
            for (int k = 0; k < 16; ++k) t.w[v][16 * (I & 3) + k] |= (uint32_t)slot[I][k] << (8 * (I >> 2));
        t.peak[v] = peak;
        t.top[v] = top;
    }
    return t;
}
constexpr P3SlotPack kP3Slots = p3_make_slots();
static_assert(kP3Slots.peak[3] == P3_POOL && kP3Slots.peak[2] <= P3_POOL, "pool size");
static_assert(kP3Slots.peak[1] == P3_POOL_128 && kP3Slots.top[1] < P3_POOL_128 && kP3Slots.top[0] < P3_POOL_128,
              "pool size, m <= 128");
__device__ const P3SlotPack p3_slot_pack = kP3Slots;

// Slot of tile (I, k); tab is this lane's dword of the packed table (I, k uniform).
__device__ inline int p3_slot(uint32_t tab, int I, int k) {
    const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)tab, ((I & 3) << 4) | k);
    return (int)((v >> ((I >> 2) << 3)) & 0xffu);
}

// The panel wavefronts' work in the phases of potrf3, for the slots s >= S0
// (tiles I = 3s + w): every slot runs the same instructions, so there is one
// basic block per step whatever the slot count; a slot past the last tile
// (I >= np) works on a clamped copy, and a slot with nothing to do works on
// whatever its indices give, and neither stores anything.

// L_Ip^T = Y C_Ip^T for one tile I > p, in place in the pool (the wavefront
// reads the whole tile before it writes it) and to global memory
// (device-coherent stores: a concurrent TRSM reads them).
template <int NPOOL>
__device__ inline void p3_solve_tile(P3SmemT<NPOOL>& sm, const double* Y, double* Mw, int ldi, uint32_t tab, int I, int p,
                                     int lane, int li, int lk) {
    double* X = sm.pool[p3_slot(tab, I, p)];
    dbl4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r)
        o = __builtin_amdgcn_mfma_f64_16x16x4f64(Y[li * P3_LD + 4 * r + lk], X[r * 64 + lane], o, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        st_coh_s(Mw, (uint32_t)((16 * I + li) + (16 * p + 4 * r + lk) * ldi), o[r]);
        X[(4 * r + lk) * 16 + li] = o[r];
    }
}

// U(p), p + 2 < np: first the solves of this wavefront's tiles I >= p+3 of
// panel p (L_Ip^T = Y C_Ip^T, in place; S(p) did only the tiles p+1 and p+2,
// which other wavefronts read); then panel p into the tiles I >= p+2 of panel
// p+1 (nxt -> pool, transposed MFMA form, for S(p+1)); then the tiles I >= p+2 of panel
// p+2: raw values from global memory into nxt (the only global reads of the
// loop, in flight during the products), reduced over the panels 0..p from the
// pool (products accumulated apart, subtracted at the end).  The panels go in
// pairs (a lone first panel when their count is odd), so the loop body is one
// basic block; the owner of tile p+2 hands its diagonal block to wavefront 0
// through Dn.
template <int S0, int NPOOL>
__device__ __forceinline__ void p3_update_slots(dbl4 (&nxt)[P3_SLOTS], P3SmemT<NPOOL>& sm, const double* Y, const double* Mc,
                                                double* Mw, int ldi, uint32_t tab, int w, int np, int p, int lane,
                                                int li, int lk) {
    constexpr int NS = P3_SLOTS - S0;
    const int c2 = 16 * (p + 2);
    const int lo = lk * 16 + li;
    int Is[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) Is[q] = imin_(P3_PW * (S0 + q) + w, np - 1);
    {
        // every slot multiplies; only the tiles I >= p+3 are stored
        double* X[NS];
        dbl4 o[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            X[q] = sm.pool[p3_slot(tab, Is[q], p)];
            o[q] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
        double yv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) yv[r] = Y[li * P3_LD + 4 * r + lk];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < NS; ++q)
                o[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(yv[r], X[q][r * 64 + lane], o[q], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int I = P3_PW * (S0 + q) + w;
            if (I >= p + 3 && I < np) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    st_coh_s(Mw, (uint32_t)((16 * I + li) + (16 * p + 4 * r + lk) * ldi), o[q][r]);
                    X[q][(4 * r + lk) * 16 + li] = o[q][r];
                }
            }
        }
    }
    {
        const double* L1 = sm.pool[p3_slot(tab, p + 1, p)];
        double av[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) av[kk] = -L1[64 * kk + lo];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int q = 0; q < NS; ++q)
                nxt[S0 + q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], sm.pool[p3_slot(tab, Is[q], p)][64 * kk + lo],
                                                                   nxt[S0 + q], 0, 0, 0);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int I = P3_PW * (S0 + q) + w;
            if (I >= p + 2 && I < np) {
                double* X = sm.pool[p3_slot(tab, I, p + 1)];
#pragma unroll
                for (int r = 0; r < 4; ++r) X[r * 64 + lane] = nxt[S0 + q][r];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) nxt[S0 + q][r] = ld_coh_s(Mc, (uint32_t)((16 * Is[q] + li) + (c2 + 4 * r + lk) * ldi));
    dbl4 red[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) red[q] = dbl4{0.0, 0.0, 0.0, 0.0};
    // operands of panel k (clamped to p: a fetch past the end is not used)
    auto fetch = [&](double (&a)[4], double (&bq)[NS][4], int k) {
        k = imin_(k, p);
        const double* A = sm.pool[p3_slot(tab, p + 2, k)];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) a[kk] = A[64 * kk + lo];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const double* B = sm.pool[p3_slot(tab, Is[q], k)];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) bq[q][kk] = B[64 * kk + lo];
        }
    };
    auto mma = [&](const double (&a)[4], const double (&bq)[NS][4]) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int q = 0; q < NS; ++q) red[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], bq[q][kk], red[q], 0, 0, 0);
    };
    double a0[4], a1[4], b0[NS][4], b1[NS][4];
    int k0 = 0;
    fetch(a0, b0, 0);
    if ((p & 1) == 0) {   // an odd panel count: panel 0 alone first
        mma(a0, b0);
        fetch(a0, b0, 1);
        k0 = 1;
    }
    fetch(a1, b1, k0 + 1);
    for (int k = k0; k <= p; k += 2) {
        mma(a0, b0);
        fetch(a0, b0, k + 2);
        mma(a1, b1);
        fetch(a1, b1, k + 3);
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        nxt[S0 + q] -= red[q];
        if (P3_PW * (S0 + q) + w == p + 2) {
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Dn[(p + 2) & 1][(4 * r + lk) * P3_LD + li] = nxt[S0 + q][r];
        }
    }
}

// p3_update_slots<s0> for a run-time s0 < P3_SLOTS.
template <int S0 = 0, int NPOOL>
__device__ __forceinline__ void p3_update_dispatch(int s0, dbl4 (&nxt)[P3_SLOTS], P3SmemT<NPOOL>& sm, const double* Y,
                                                   const double* Mc, double* Mw, int ldi, uint32_t tab, int w, int np,
                                                   int p, int lane, int li, int lk) {
    if constexpr (S0 == P3_SLOTS - 1) {
        p3_update_slots<S0>(nxt, sm, Y, Mc, Mw, ldi, tab, w, np, p, lane, li, lk);
    } else {
        if (s0 == S0) p3_update_slots<S0>(nxt, sm, Y, Mc, Mw, ldi, tab, w, np, p, lane, li, lk);
        else p3_update_dispatch<S0 + 1>(s0, nxt, sm, Y, Mc, Mw, ldi, tab, w, np, p, lane, li, lk);
    }
}

// The raw tiles are read with device-coherent loads: in the single-launch
// factor the previous tile column's updates are other workgroups' stores.
// In-place Cholesky of the m x m lower triangle of M (column-major, leading
// dimension ld), m a multiple of 64, m <= 256; zeros go only into the upper
// parts of the diagonal 16 x 16 blocks (the rest of the strict upper triangle
// is left as it is, for the caller to clear off the dependency chain).
// Yd + 256 p: Y_p = L_pp^{-1}, the inverse of the p-th 16 x 16 diagonal block
// (column-major, upper part 0).  Thread 0 returns the first failing local
// column (or -1) and the log det pair.
//
// Panels are announced as they are finished (fpo == nullptr: never, a test
// hook of the caller): *fpo is raised by one for each
// (agent-scope relaxed atomic add), once the off-diagonal tiles L_Ip (I > p)
// and Y_p are in global memory, written with device-coherent stores, so a
// kernel running concurrently on other compute units may read them with
// device-coherent loads as soon as it sees *fpo > p.  (Panel p is announced
// at the end of U(p), when its stores have long completed; the last one at
// the end.)
//
// Software pipeline over the 16-column panels p, two phases per panel:
//   S(p): L_pp and Y_pp go out; the tiles (p+1, p) and (p+2, p), which other
//         wavefronts need next, are solved (L_Ip = C_Ip Y^T) in place in the
//         LDS pool and to global memory by their owners;
//   U(p): wavefront 0 forms the next diagonal block D_{p+1} = Dn - L_{p+1,p}
//         L_{p+1,p}^T and factors it (factor16), while the panel wavefronts solve
//         their other tiles of panel p, add panel p into the tiles of panel
//         p+1 (into the pool, solved from S(p+1) on) and reduce the tiles of
//         panel p+2 over panels 0..p; the
//         owner of tile p+2 hands its diagonal block to wavefront 0 through Dn
//         (by parity).  Y_p and Y_{p+1} live in two LDS buffers (by parity):
//         the panel wavefronts' solves of panel p in U(p) still read Y_p while
//         wavefront 0 writes Y_{p+1}.
// Every tile of L stays in the LDS pool from its reduction to its last use,
// so global memory is read only for the raw tiles, each once.  The chain of
// diagonal factorizations overlaps all the other work.
template <int NPOOL>
__device__ inline void potrf3(double* M, int64_t ld, int m, double* Yd, P3SmemT<NPOOL>& sm, int* fail_out, double* ls_out,
                              double* lc_out, int* fpo) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    // np and ldi opaque here: the offsets derived from them are formed in this
    // task, not hoisted to the start of a kernel that runs other tasks too
    // (where they would only occupy registers)
    int np = m / 16, ldi = (int)ld;
    asm volatile("" : "+s"(np), "+s"(ldi));
    const double* Mc = uniform_ptr(M);   // with unsigned 32-bit offsets: scalar base + vector offset loads
    double* Mw = (double*)Mc;
    int fail = -1;
    const uint32_t tab = p3_slot_pack.w[np / 4 - 1][lane];
    // panel 0 into the pool, transposed MFMA form: [r*64 + lane] = C[16I + li][4r + lk];
    // D_0 = tile (0, 0); Y's upper part stays 0 from here on
    if (w < 4) {   // 256 threads: one element of each 16 x 16 tile each
        double v[16];
        const int q = threadIdx.x, r = q >> 6, ln = q & 63;
#pragma unroll
        for (int I = 0; I < 16; ++I)
            v[I] = ld_coh_s(Mc, (uint32_t)((16 * imin_(I, np - 1) + (ln & 15)) + (4 * r + (ln >> 4)) * ldi));
#pragma unroll
        for (int I = 1; I < 16; ++I)
            if (I < np) sm.pool[p3_slot(tab, I, 0)][q] = v[I];
        // D_0 symmetric from the lower triangle of the tile
        const int i = threadIdx.x & 15, j = threadIdx.x >> 4;
        sm.D[j * P3_LD + i] = ld_coh_s(Mc, (uint32_t)(imax_(i, j) + imin_(i, j) * ldi));
    }
    for (int e = threadIdx.x; e < 2 * 16 * P3_LD; e += 256) sm.Y[0][e] = 0.0;
    // panel wavefronts w = 1..P3_PW own the row tiles I = P3_PW s + w >= 1 of every panel
    dbl4 nxt[P3_SLOTS];
    // raw tiles of panel 1 (nothing to reduce yet); tile 1 is owned by
    // wavefront 1, slot 0, and goes to Dn
    if (w != 0) {
#pragma unroll
        for (int s = 0; s < P3_SLOTS; ++s) {
            const int I = imin_(P3_PW * s + w, np - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) nxt[s][r] = ld_coh_s(Mc, (uint32_t)((16 * I + li) + (16 + 4 * r + lk) * ldi));
        }
        if (w == 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Dn[1][(4 * r + lk) * P3_LD + li] = nxt[0][r];
        }
    }
    __syncthreads();
    if (w == 0) p3_factor16(sm, sm.Y[0], 0, fail);
    p3_bar_lds();
    for (int p = 0; p < np; ++p) {
        const int c0 = 16 * p;
        // ---- S(p)
        if (w == 0) {
            double* Yg = (double*)uniform_ptr(Yd + (int64_t)p * 256);
            double dv[4], yv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = lane & 15, j = (lane >> 4) + 4 * q;
                dv[q] = (j <= i) ? sm.D[j * P3_LD + i] : 0.0;
                yv[q] = sm.Y[p & 1][i * P3_LD + j];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = lane & 15, j = (lane >> 4) + 4 * q;
                st_s(Mw, (uint32_t)((c0 + i) + (c0 + j) * ldi), dv[q]);
                st_coh_s(Yg, (uint32_t)(i + 16 * j), yv[q]);
            }
        } else {
            // the tiles other wavefronts read in U(p): (p+1, p) and (p+2, p)
            // (each owned by a different wavefront); the rest waits for U(p)
            const double* Yp = sm.Y[p & 1];
            if (p + 1 < np && ((p + 1) - w) % P3_PW == 0) p3_solve_tile(sm, Yp, Mw, ldi, tab, p + 1, p, lane, li, lk);
            if (p + 2 < np && ((p + 2) - w) % P3_PW == 0) p3_solve_tile(sm, Yp, Mw, ldi, tab, p + 2, p, lane, li, lk);
        }
        p3_bar_lds();   // panel p of L in the pool (the global stores stay in flight)
        if (p + 1 == np) break;
        // ---- U(p)
        if (w == 0) {
            // D_{p+1} = Dn - L_{p+1,p} L_{p+1,p}^T, then its factorization
            dbl4 acc;
            const double* L1 = sm.pool[p3_slot(tab, p + 1, p)];
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = sm.Dn[(p + 1) & 1][(4 * r + lk) * P3_LD + li];
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const double v = L1[(kk + lk) * 16 + li];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-v, v, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.D[(4 * r + lk) * P3_LD + li] = acc[r];
            // the upper triangle mirrored from the lower one (p3_factor16 reads both)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (li > 4 * r + lk) sm.D[li * P3_LD + 4 * r + lk] = acc[r];
            p3_wsync();
            p3_factor16(sm, sm.Y[(p + 1) & 1], c0 + 16, fail);
        } else if (p + 2 < np) {
            // slots s >= s0 hold the tiles I >= p+2
            const int s0 = imin_(P3_SLOTS - 1, imax_(0, (p + 2 - w + P3_PW - 1) / P3_PW));
            p3_update_dispatch(s0, nxt, sm, sm.Y[p & 1], Mc, Mw, ldi, tab, w, np, p, lane, li, lk);
        }
        // D, Y of p+1; panel p+1 in the pool; Dn; and the stores of panel p
        // complete, so it is announced.
        p3_bar_all();
        if (threadIdx.x == 0 && fpo) add_coh_i(fpo, 1);
    }
    p3_bar_all();   // the last panel's stores complete
    if (threadIdx.x == 0 && fpo) add_coh_i(fpo, 1);
    // log det: 2 log L_jj in parallel, then a fixed-order compensated sum
    // (lane l of wavefront 0 sums entries l, l+64, ..., then the lanes are
    // joined pairwise by a butterfly)
    for (int t = threadIdx.x; t < m; t += 256) sm.dg[t] = 2.0 * log(sm.dg[t]);
    __syncthreads();
    if (w == 0) {
        double ps = 0.0, pc = 0.0;
        for (int t = lane; t < m; t += 64) neumaier(ps, pc, sm.dg[t]);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double qs = __shfl_xor(ps, o), qc = __shfl_xor(pc, o);
            // the lower lane of each pair is the left operand, so both lanes agree
            const bool lo = (lane & o) == 0;
            const double a = lo ? ps : qs, b = lo ? qs : ps;
            const double t = a + b;
            const double e = (fabs(a) >= fabs(b)) ? (a - t) + b : (b - t) + a;
            pc = (lo ? pc + qc : qc + pc) + e;
            ps = t;
        }
        if (lane == 0) {
            *fail_out = fail;
            *ls_out = ps;
            *lc_out = pc;
        }
    }
}
