// Cholesky of one diagonal tile (m <= 256, m a multiple of 64) by one
// workgroup of 1 + P3_PW wavefronts, left-looking over 16-column panels with a
// one-panel lookahead:
//   - wavefronts 1..P3_PW own the 16 x 16 row tiles I = w, w+P3_PW, ... of every
//     panel; the reduced current panel sits in LDS in transposed MFMA form
//     (lane (i, k) reads C[16I + i][c0 + 4r + k], the layout the matrix cores
//     take as the B operand, so the panel solve needs no shuffle);
//   - the diagonal 16 x 16 block is factored by wavefront 0 (two 8 x 8
//     Cholesky factorizations and inverses kept in registers, redundantly in
//     every lane, joined by an 8 x 8 TRSM and SYRK), while the other
//     wavefronts reduce the panels ahead of it (see potrf3 below);
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
#define P3_POOL 65   // 16 x 16 tiles of L alive at once at m = 256 (checked by p3_make_slots)

struct P3Smem {
    double D[16 * P3_LD];          // diagonal block of the current panel, D(i, j) at D[j * P3_LD + i]
    double Y[2][16 * P3_LD];       // Y_p = L_pp^{-1} in Y[p & 1], Y(i, j) at [i * P3_LD + j]: the panel
                                   // wavefronts still read Y_p while wavefront 0 forms Y_{p+1}
    double S22[8 * 9];             // factor16 scratch: S(i, j) at S22[i * 9 + j]
    double T[8 * 9];               // T = L21 Y11, T(i, j) at T[i * 9 + j]
    double Dn[2][16 * P3_LD];      // next diagonal blocks (by parity), reduced up to two panels back
    double pool[P3_POOL][256];     // tiles (I, k) of L in slots given by p3_slot: first the reduced tile in
                                   // transposed MFMA form (r * 64 + lane), then, solved in place,
                                   // L[16I + i][16k + j] at [j * 16 + i]
    double dg[256];                // diagonal of L, then 2 log L_jj
    double ps[64], pc[64];         // log det partial sums
    double lsum, lcomp;
    int fail;
};

// Packed lower triangle of an 8 x 8 matrix, by columns.
#define P8(i, j) ((j) * 8 - ((j) * ((j) - 1)) / 2 + ((i) - (j)))

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

// In-register Cholesky of the packed 8 x 8 lower triangle a; rinv[j] = 1/L_jj.
// (The logarithms of the pivots are taken after the sweep, off this chain.)
// *fail gets the first local column (base + j) whose pivot is not positive.
__device__ inline void p3_chol8(double (&a)[36], double (&rinv)[8], int base, int& fail) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const double piv = a[P8(j, j)];
        if (!(piv > 0.0) && fail < 0) fail = base + j;
        double s, r;
        p3_sqrt_rsqrt(piv, s, r);
        a[P8(j, j)] = s;
        rinv[j] = r;
#pragma unroll
        for (int i = j + 1; i < 8; ++i) a[P8(i, j)] *= r;
#pragma unroll
        for (int k = j + 1; k < 8; ++k)
#pragma unroll
            for (int i = k; i < 8; ++i) a[P8(i, k)] = fma(-a[P8(i, j)], a[P8(k, j)], a[P8(i, k)]);
    }
}

// In place: the packed 8 x 8 lower-triangular L becomes L^{-1} (rinv = 1/L_jj).
// Column j is done top down; y_ij needs L_ik (k >= j, columns not yet
// replaced, and L_ij itself still in place) and y_kj (k < i, already there).
__device__ inline void p3_inv8(double (&a)[36], const double (&rinv)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
#pragma unroll
        for (int i = j + 1; i < 8; ++i) {
            double s = a[P8(i, j)] * rinv[j];
#pragma unroll
            for (int k = j + 1; k < i; ++k) s = fma(a[P8(i, k)], a[P8(k, j)], s);
            a[P8(i, j)] = -s * rinv[i];
        }
        a[P8(j, j)] = rinv[j];
    }
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

// Store a packed 8 x 8 lower triangle (identical in every lane) into LDS
// from lane 0, at compile-time addresses.  ToY: into Y ([row][col]) at
// block offset o; otherwise into sm.D ([col][row]), the diagonal also into
// sm.dg.
template <bool ToY>
__device__ inline void p3_put8(P3Smem& sm, double* Y, const double (&l)[36], int o, int base) {
    if ((threadIdx.x & 63) != 0) return;
#pragma unroll
    for (int jj = 0; jj < 8; ++jj)
#pragma unroll
        for (int ii = jj; ii < 8; ++ii) {
            const int e = P8(ii, jj);
            if (ToY) {
                Y[(o + ii) * P3_LD + o + jj] = l[e];
            } else {
                sm.D[(o + jj) * P3_LD + o + ii] = l[e];
                if (ii == jj) sm.dg[base + o + ii] = l[e];
            }
        }
}

// Factor the 16 x 16 block in sm.D (lower part) on one wavefront: L_pp back
// into the lower part of sm.D ([col][row]; the upper part is left as is) and
// Y = L_pp^{-1} into the lower part of Y ([row][col]; its upper part is
// zero from the start).  With D = [D11 .; D21 D22] (8 x 8 blocks):
// L11 = chol(D11), L21 = D21 L11^{-T} (row by row), S = D22 - L21 L21^T,
// L22 = chol(S), and Y = [Y11 0; -Y22 L21 Y11  Y22].
__device__ inline void p3_factor16(P3Smem& sm, double* Y, int base, int& fail) {
    const int lane = threadIdx.x & 63;
    double a[36], r[8], l21[8];
    // 1. L11 = chol(D11), in every lane; lane i < 8 forms row i of L21 (in place in sm.D)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int i = j; i < 8; ++i) a[P8(i, j)] = sm.D[j * P3_LD + i];
    p3_chol8(a, r, base, fail);
    if (lane < 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            double v = sm.D[j * P3_LD + 8 + lane];
#pragma unroll
            for (int k = 0; k < j; ++k) v = fma(-l21[k], a[P8(j, k)], v);
            l21[j] = v * r[j];
            sm.D[j * P3_LD + 8 + lane] = l21[j];
        }
    }
    // 2. Y11 = L11^{-1} (in place); T = L21 Y11 (row i on lane i < 8)
    p3_put8<false>(sm, Y, a, 0, base);
    p3_inv8(a, r);
    p3_put8<true>(sm, Y, a, 0, base);
    if (lane < 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            double v = 0.0;
#pragma unroll
            for (int k = j; k < 8; ++k) v = fma(l21[k], a[P8(k, j)], v);
            sm.T[lane * 9 + j] = v;
        }
    }
    p3_wsync();
    // 3. S = D22 - L21 L21^T, lane (i, j), j <= i
    {
        const int i = lane >> 3, jj = lane & 7;
        if (jj <= i) {
            double v = sm.D[(8 + jj) * P3_LD + 8 + i];
#pragma unroll
            for (int k = 0; k < 8; ++k) v = fma(-sm.D[k * P3_LD + 8 + i], sm.D[k * P3_LD + 8 + jj], v);
            sm.S22[i * 9 + jj] = v;
        }
    }
    p3_wsync();
    // 4. L22 = chol(S), Y22 = L22^{-1}, in every lane
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int i = j; i < 8; ++i) a[P8(i, j)] = sm.S22[i * 9 + j];
    p3_chol8(a, r, base + 8, fail);
    p3_put8<false>(sm, Y, a, 8, base);
    p3_inv8(a, r);
    p3_put8<true>(sm, Y, a, 8, base);
    // 5. Y21 = -Y22 T, column j on lane j < 8
    if (lane < 8) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) t[k] = sm.T[k * 9 + lane];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k <= i; ++k) v = fma(a[P8(i, k)], t[k], v);
            Y[(8 + i) * P3_LD + lane] = -v;
        }
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
        for (int I = 1; I < np; ++I) { slot[I][0] = fr[--nf]; ++live; }
        peak = live;
        for (int p = 0; p + 1 < np; ++p) {
            for (int I = p + 2; I < np; ++I) { slot[I][p + 1] = fr[--nf]; ++live; }
            if (live > peak) peak = live;
            if (p + 2 < np)
                for (int k = 0; k <= p; ++k) { fr[nf++] = slot[p + 2][k]; --live; }
            fr[nf++] = slot[p + 1][p];
            --live;
        }
        for (int I = 0; I < 16; ++I)
            for (int k = 0; k < 16; ++k) t.w[v][16 * (I & 3) + k] |= (uint32_t)slot[I][k] << (8 * (I >> 2));
        t.peak[v] = peak;
    }
    return t;
}
constexpr P3SlotPack kP3Slots = p3_make_slots();
static_assert(kP3Slots.peak[3] == P3_POOL && kP3Slots.peak[2] <= P3_POOL, "pool size");
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
__device__ inline void p3_solve_tile(P3Smem& sm, const double* Y, double* Mw, int ldi, uint32_t tab, int I, int p,
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
template <int S0>
__device__ __forceinline__ void p3_update_slots(dbl4 (&nxt)[P3_SLOTS], P3Smem& sm, const double* Y, const double* Mc,
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
template <int S0 = 0>
__device__ __forceinline__ void p3_update_dispatch(int s0, dbl4 (&nxt)[P3_SLOTS], P3Smem& sm, const double* Y,
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
__device__ inline void potrf3(double* M, int64_t ld, int m, double* Yd, P3Smem& sm, int* fail_out, double* ls_out,
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
        const int i = threadIdx.x & 15, j = threadIdx.x >> 4;
        sm.D[j * P3_LD + i] = ld_coh_s(Mc, (uint32_t)(i + j * ldi));
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
