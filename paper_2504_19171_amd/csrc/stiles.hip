// HIP kernels and the C ABI (include/stiles.h) of the band-plus-arrowhead
// selected inversion: tile Cholesky with log det, then Phase 1 and Phase 2 of
// the two-phase backward recurrence (arXiv 2504.19171, Sec. III-D).
//
// Execution: every step is enqueued on the caller's stream; each kernel below
// covers one tile-level operation over all the tiles it can do at once.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/stiles.h"
#include "common.hpp"
#include "gemm_block.hpp"
#include "tile_ops.hpp"
#include "persist.hpp"
#include "wave_gemm.hpp"
#include "potrf3.hpp"

#define NT 256
#define WS_HEAD 256  // bytes reserved at the start of every workspace (info and scheduler words)

// ---------------------------------------------------------------------------
// Layout
// ---------------------------------------------------------------------------
static int make_layout(int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile, stiles_layout* o) {
    if (n < 1) return -1;
    if (bandwidth < 0) return -2;
    if (arrow < 0 || arrow >= n || arrow > 512) return -3;
    if (!(tile == 64 || tile == 128 || tile == 192 || tile == 256)) return -4;
    memset(o, 0, sizeof(*o));
    o->n = n; o->bandwidth = bandwidth; o->arrow = arrow; o->tile = tile;
    o->nb = n - arrow;
    o->w = std::min<int64_t>(bandwidth, o->nb - 1);
    o->nt = (o->nb + tile - 1) / tile;
    int64_t bt = (o->w + tile - 1) / tile;
    if (bt > o->nt - 1) bt = o->nt - 1;
    o->bt = (int32_t)bt;
    o->arrow_ld = (int32_t)((arrow + 15) / 16 * 16);
    const int64_t b2 = (int64_t)tile * tile;
    o->off_band = 0;
    o->off_arrow = o->nt * (o->bt + 1) * b2;
    o->off_corner = o->off_arrow + o->nt * (int64_t)o->arrow_ld * tile;
    o->total_doubles = o->off_corner + (int64_t)o->arrow_ld * o->arrow_ld;
    return 0;
}

// Parts of the Phase 2 sums: two (measured: as fast as three at tile 256,
// faster at 128 and, by a fifth in the batched form, at 64, where the extra
// tasks of the three-part form cost more than the shorter chain saves).
// STILES_P2_SPLIT=3 selects the three-part form (measurement and tests).
static int p2_split_for(int tile) {
    (void)tile;
    if (const char* e = getenv("STILES_P2_SPLIT")) {
        const int v = atoi(e);
        if (v == 2 || v == 3) return v;
    }
    return 2;
}

static Lay to_dev(const stiles_layout& s) {
    Lay l;
    l.nb = s.nb; l.w = s.w; l.nt = s.nt;
    l.off_band = s.off_band; l.off_arrow = s.off_arrow; l.off_corner = s.off_corner;
    l.total = s.total_doubles;
    l.b = s.tile; l.bt = s.bt; l.ap = s.arrow_ld; l.a = (int)s.arrow;
    l.p2s = p2_split_for(s.tile);
    return l;
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void k_zero_ints(int* p, int64_t n) {
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x; i < n; i += (int64_t)blockDim.x * gridDim.x) p[i] = 0;
}
__global__ void k_set_int(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Pack the canonical band form into the tile layout (every double written).
// Workgroup g < N (B+1) writes band tile g = J (B+1) + d, i.e. tile (J+d, J);
// the next N write the arrow tiles J; the last one the corner.
//
// A band tile is written 32 columns at a time through LDS.  Column c of tile
// (J+d, J) holds A[(J+d) b + r, J b + c]; in the band form that is
// ab[d b + r - c, J b + c] (on and below the diagonal) and ab[c - r, J b + r]
// (above it, diagonal tiles only).  For a fixed band-form row k both are 32
// consecutive doubles over the 32 columns, so the reads run along the rows of
// ab, the block is assembled in LDS and written out column by column: both
// sides coalesced.  The arrow tiles go the same way: a row of P is contiguous,
// a tile column is contiguous.
#define PACK_CB 32
#define PACK_RB 256
#define PACK_SMEM_DOUBLES (PACK_CB * (PACK_RB + 1))
#define PACK_U 8   // loads in flight per thread
__global__ __launch_bounds__(NT) void k_pack(const double* __restrict__ ab, const double* __restrict__ P,
                                            const double* __restrict__ C, double* __restrict__ T, Lay L) {
    __shared__ double blk[PACK_SMEM_DOUBLES];   // [c][r]: column c at c * b (band) or c * (rows + 1) (arrow)
    const int b = L.b;
    const int64_t nband = L.nt * (int64_t)(L.bt + 1);
    const int64_t g = blockIdx.x;
    const int tid = threadIdx.x;
    if (g < nband) {
        const int64_t J = g / (L.bt + 1);
        const int d = (int)(g % (L.bt + 1));
        double* O = T + g * (int64_t)b * b;
        const bool live = J + d < L.nt;
        const int64_t i0 = (J + d) * b, j0 = J * b;   // global row / column of the tile's (0, 0)
        if (b == 64) {
            // 64 x 64 tiles: the staging costs more than it saves (each block
            // would read 95 band-form rows for 64 tile rows); thread t writes
            // row t % 64 of columns t / 64, t / 64 + 4, ...
            // (every load from a valid address, the unused ones dropped: a
            // load under a branch would wait before the next one issues)
            const int r = tid % 64;
            const int64_t i = i0 + r;
            constexpr int NQ = 64 / (NT / 64);
            double v[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int64_t j = j0 + tid / 64 + q * (NT / 64);
                const int64_t k = i >= j ? i - j : j - i, lo = i >= j ? j : i;
                const bool ok = live && i < L.nb && j < L.nb && k <= L.w;
                v[q] = ab[ok ? k * L.nb + lo : 0];
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int c = tid / 64 + q * (NT / 64);
                const int64_t j = j0 + c;
                const bool in = live && i < L.nb && j < L.nb;
                const int64_t k = i >= j ? i - j : j - i;
                O[r + c * 64] = (in && k <= L.w) ? v[q] : ((live && !in && i == j) ? 1.0 : 0.0);
            }
            return;
        }
        for (int cb = 0; cb < b; cb += PACK_CB) {
            // defaults: 0, or 1 on the diagonal past the band part (identity padding)
            for (int e = tid; e < PACK_CB * b; e += NT) {
                const int c = e / b, r = e % b;
                blk[e] = (live && d == 0 && r == cb + c && i0 + r >= L.nb) ? 1.0 : 0.0;
            }
            __syncthreads();
            if (live) {
                // on and below the diagonal: k = d b + r - c', c' = cb + c.
                // PACK_U loads per thread are issued before their LDS stores,
                // each from a valid address (the unused ones dropped): a load
                // under a branch would wait before the next one issues.
                const int klo = imax_(0, d * b - cb - (PACK_CB - 1)), khi = imin_((int)L.w, d * b + b - 1 - cb);
                const int n = (khi - klo + 1) * PACK_CB;
                for (int e0 = tid; e0 < n; e0 += NT * PACK_U) {
                    double v[PACK_U];
                    int at[PACK_U];
#pragma unroll
                    for (int q = 0; q < PACK_U; ++q) {
                        const int e = e0 + q * NT;
                        const int k = klo + e / PACK_CB, c = e % PACK_CB;
                        const int r = k - d * b + cb + c;
                        const int64_t j = j0 + cb + c;
                        const bool ok = e < n && r >= 0 && r < b && i0 + r < L.nb && j < L.nb;
                        v[q] = ab[ok ? (int64_t)k * L.nb + j : 0];
                        at[q] = ok ? c * b + r : -1;
                    }
#pragma unroll
                    for (int q = 0; q < PACK_U; ++q)
                        if (at[q] >= 0) blk[at[q]] = v[q];
                }
                if (d == 0) {
                    // above the diagonal: k = c' - r >= 1, value ab[k, j0 + r]
                    const int khi2 = imin_((int)L.w, cb + PACK_CB - 1);
                    const int n2 = imax_(khi2, 0) * PACK_CB;
                    for (int e0 = tid; e0 < n2; e0 += NT * PACK_U) {
                        double v[PACK_U];
                        int at[PACK_U];
#pragma unroll
                        for (int q = 0; q < PACK_U; ++q) {
                            const int e = e0 + q * NT;
                            const int k = 1 + e / PACK_CB, c = e % PACK_CB;
                            const int r = cb + c - k;
                            const bool ok = e < n2 && r >= 0 && j0 + cb + c < L.nb;
                            v[q] = ab[ok ? (int64_t)k * L.nb + j0 + r : 0];
                            at[q] = ok ? c * b + r : -1;
                        }
#pragma unroll
                        for (int q = 0; q < PACK_U; ++q)
                            if (at[q] >= 0) blk[at[q]] = v[q];
                    }
                }
            }
            __syncthreads();
            for (int e = tid; e < PACK_CB * b; e += NT) O[(int64_t)cb * b + e] = blk[e];
            __syncthreads();
        }
    } else if (g < nband + L.nt) {
        const int64_t J = g - nband;
        double* O = T + L.arrow(J);
        const int ap = L.ap;
        const int64_t j0 = J * b;
        for (int cb = 0; cb < b; cb += PACK_CB) {
            for (int rb = 0; rb < ap; rb += PACK_RB) {
                const int nr = imin_(PACK_RB, ap - rb);
                // rows r of P over the block's 32 columns (contiguous), into [c][r]
                for (int e0 = tid; e0 < nr * PACK_CB; e0 += NT * PACK_U) {
                    double v[PACK_U];
                    int at[PACK_U];
                    bool ok[PACK_U];
#pragma unroll
                    for (int q = 0; q < PACK_U; ++q) {
                        const int e = e0 + q * NT;
                        const int r = e / PACK_CB, c = e % PACK_CB;
                        const int64_t j = j0 + cb + c;
                        ok[q] = rb + r < L.a && j < L.nb;
                        v[q] = P[ok[q] ? (int64_t)(rb + r) * L.nb + j : 0];
                        at[q] = e < nr * PACK_CB ? c * (nr + 1) + r : -1;
                    }
#pragma unroll
                    for (int q = 0; q < PACK_U; ++q)
                        if (at[q] >= 0) blk[at[q]] = ok[q] ? v[q] : 0.0;
                }
                __syncthreads();
                for (int e = tid; e < nr * PACK_CB; e += NT) {
                    const int c = e / nr, r = e % nr;
                    O[(int64_t)(cb + c) * ap + rb + r] = blk[c * (nr + 1) + r];
                }
                __syncthreads();
            }
        }
    } else {
        double* O = T + L.corner();
        const int ap = L.ap;
        for (int e = tid; e < ap * ap; e += NT) {
            const int r = e % ap, c = e / ap;
            O[e] = (r < L.a && c < L.a) ? C[r * L.a + c] : (r == c ? 1.0 : 0.0);
        }
    }
}

// Zero the band tiles (J+d, J) with J+d >= N (outside the matrix); block bid
// of nblk.
__device__ inline void zero_unused_body(double* T, const Lay& L, int bid, int nblk) {
    const int64_t b2 = (int64_t)L.b * L.b;
    const int64_t ntail = (int64_t)L.bt * (L.bt + 1) / 2;  // tiles J+d >= N
    const int64_t tot = ntail * b2;
    for (int64_t idx = bid * (int64_t)NT + threadIdx.x; idx < tot; idx += (int64_t)nblk * NT) {
        const int64_t t = idx / b2, e = idx % b2;
        // enumerate (J, d) with J = N-1-m, d = m+1..B, m = 0..B-1
        int64_t m = 0, cnt = t;
        while (cnt >= L.bt - m) { cnt -= L.bt - m; ++m; }
        const int64_t J = L.nt - 1 - m, d = m + 1 + cnt;
        T[L.band(J, (int)d) + e] = 0.0;
    }
}
__global__ __launch_bounds__(NT) void k_zero_unused(double* T, Lay L) { zero_unused_body(T, L, blockIdx.x, gridDim.x); }

// ---------------------------------------------------------------------------
// Factor kernels
// ---------------------------------------------------------------------------

// POTRF of one m x m diagonal block (m <= 256), optional TRTRI of the result
// into X, log det partial into ldp[0..1], first failing column into *info
// (atomicMin of the 1-based global column col_base + c + 1).
__device__ __forceinline__ void potrf_body(double* M, int64_t ld, int m, double* X, int64_t ldx, double* ldp, int* info,
                                  int64_t col_base, double* smem) {
    // device memory (a batched caller reads these pointers from its table)
    M = (double*)(GLOBAL_AS double*)M;
    if (X) X = (double*)(GLOBAL_AS double*)X;
    int fail;
    double s, c;
    potrf_tile(M, ld, m, smem, &fail, &s, &c);
    if (threadIdx.x == 0) {
        ldp[0] = s;
        ldp[1] = c;
        if (fail >= 0) atomicMin(info, (int)(col_base + fail + 1));
    }
    if (X) {
        __syncthreads();
        int bad;
        trtri_tile(M, ld, X, ldx, m, smem, &bad);
    }
}
__global__ __launch_bounds__(NT) void k_potrf(double* M, int64_t ld, int m, double* X, int64_t ldx,
                                             double* ldp, int* info, int64_t col_base) {
    extern __shared__ double smem[];
    potrf_body(M, ld, m, X, ldx, ldp, info, col_base, smem);
}

// In place: columns are produced last block first, so every column block
// read later is still unmodified (X^T is upper triangular).
__device__ inline void trsm_rows(double* C, int64_t ld, int valid, const double* X, int64_t ldx,
                                 int ncols, double* smem) {
    for (int cb = ncols / 64 - 1; cb >= 0; --cb) {
        GAcc g;
        gacc_zero(g);
        gemm_acc(g, opnd(C, ld, 0, valid), opnd(X + cb * 64, ldx, 1, 64), (cb + 1) * 64, smem);
        gemm_store(g, smem, 1.0, 0.0, nullptr, 0, C + (int64_t)cb * 64 * ld, ld, valid, 64);
    }
}

// Generic TRSM on a contiguous row panel (used for the blocked corner).
__global__ __launch_bounds__(NT) void k_trsm_generic(double* C, int64_t ld, int rows, const double* X,
                                                    int64_t ldx, int ncols) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    const int rb = blockIdx.x;
    trsm_rows(C + rb * 64, ld, imin_(64, rows - rb * 64), X, ldx, ncols, smem);
}

// ---------------------------------------------------------------------------
// Factor kernels of the band tile columns
// ---------------------------------------------------------------------------

// Strict upper triangles of the band diagonal tiles set to 0 (the layout's
// convention for L; the diagonal-tile POTRF leaves them, as nothing in the
// factorization reads them).  Eight workgroups per tile, b/8 columns each.
__device__ inline void zero_upper_body(double* Lm, const Lay& L, int bid) {
    const int64_t J = bid >> 3;
    const int cw = L.b / 8, c0 = (bid & 7) * cw;
    double* T = Lm + L.band(J, 0);
    for (int c = c0; c < c0 + cw; ++c)
        for (int i = threadIdx.x; i < c; i += NT) T[i + (int64_t)c * L.b] = 0.0;
}
__global__ __launch_bounds__(NT) void k_zero_upper(double* Lm, Lay L) { zero_upper_body(Lm, L, blockIdx.x); }

// Panel TRSM of one 16-row block C (16 x b, leading dimension ld), R = C
// L_JJ^{-T} in place, one 16-column panel p per step:
//   Z_p = C_p - sum_{p' < p} R_p' L_{p,p'}^T,   R_p = Z_p Y_p^T   (Y_p = L_pp^{-1}),
// with the transposed products on the matrix cores (Z_p^T = C_p^T - L_{p,p'}
// R_p'^T, R_p^T = Y_p Z_p^T) so every global access runs down a column.  The
// reduction of a step is spread over the 4 wavefronts (panels p' = w, w+4,
// ... of wavefront w) and summed in LDS in a fixed order; the tiles L_{p,p'}
// of the next step are loaded while the current one is multiplied.  R stays in
// LDS ([column][row]) and is zero where not yet computed, so a product with a
// panel that is not there yet adds nothing and the loop has no branches.
//
// Concurrent mode (fpo != nullptr): L_JJ is being factored (potrf3) at the
// same time; step p waits until *fpo > p, reads L and Y with device-coherent
// loads, writes R with device-coherent stores and raises *ftr after each step.
#define TR_LD 16
struct TrSmem {
    double R[256 * TR_LD];
    double P[4][256];
    int sh;
};
__device__ inline bool tr_panel(double* C, int ld, const double* Ljj, const double* Yd, int b, const int* fpo,
                                int* ftr, const Sched& sc, TrSmem& sm, int ticket) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int np = b / 16;
    const bool coh = fpo != nullptr;
    C = (double*)uniform_ptr(C);
    Ljj = uniform_ptr(Ljj);
    Yd = uniform_ptr(Yd);
    for (int e = threadIdx.x; e < b * TR_LD; e += blockDim.x) sm.R[e] = 0.0;
    auto ldL = [&](uint32_t idx) { return coh ? ld_coh_s(Ljj, idx) : ld_s(Ljj, idx); };
    // A operands of step s for this wavefront: -L_{s,p'} for p' = w + 4t (the
    // tile column clamped into the finished part; its product is then with a
    // zero panel of R)
    auto fetchA = [&](double (&a)[4][4], int s) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int pa = imax_(0, imin_(w + 4 * t, s - 1));
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) a[t][kk] = -ldL((uint32_t)((16 * s + li) + (16 * pa + 4 * kk + lk) * b));
        }
    };
    double acur[4][4], anext[4][4];
    dbl4 cn;
#pragma unroll
    for (int r = 0; r < 4; ++r) cn[r] = coh ? ld_coh_s(C, (uint32_t)(li + (4 * r + lk) * ld)) : ld_s(C, (uint32_t)(li + (4 * r + lk) * ld));
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acur[t][kk] = 0.0;
    __syncthreads();
    for (int p = 0; p < np; ++p) {
        if (coh && !sched_wait(sc, (int*)fpo, p + 1, &sm.sh)) return false;
        // loads for this step's Y and the next step's operands (panels <= p
        // are finished, so the tiles L_{p+1,p'}, p' <= p, are there)
        double yv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t yi = (uint32_t)(p * 256 + li + 16 * (4 * r + lk));
            yv[r] = coh ? ld_coh_s(Yd, yi) : ld_s(Yd, yi);
        }
        const int pn = imin_(p + 1, np - 1);
        fetchA(anext, pn);
        dbl4 cnext;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t ci = (uint32_t)(li + (16 * pn + 4 * r + lk) * ld);
            cnext[r] = coh ? ld_coh_s(C, ci) : ld_s(C, ci);
        }
        // this wavefront's part of Z_p^T (wavefronts past the fourth, if the
        // workgroup has them, only keep the barriers)
        if (w < 4) {
            dbl4 z;
#pragma unroll
            for (int r = 0; r < 4; ++r) z[r] = (w == 0) ? cn[r] : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int p2 = imin_(w + 4 * t, np - 1);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    z = __builtin_amdgcn_mfma_f64_16x16x4f64(acur[t][kk], sm.R[(16 * p2 + 4 * kk + lk) * TR_LD + li], z,
                                                             0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.P[w][r * 64 + lane] = z[r];
        }
        __syncthreads();
        if (w == 0) {
            // Z_p^T in the D layout is the B operand of R_p^T = Y_p Z_p^T as it stands
            dbl4 zs, o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r)
                zs[r] = ((sm.P[0][r * 64 + lane] + sm.P[1][r * 64 + lane]) + sm.P[2][r * 64 + lane]) +
                        sm.P[3][r * 64 + lane];
#pragma unroll
            for (int r = 0; r < 4; ++r) o = __builtin_amdgcn_mfma_f64_16x16x4f64(yv[r], zs[r], o, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                sm.R[(16 * p + 4 * r + lk) * TR_LD + li] = o[r];
                const uint32_t ci = (uint32_t)(li + (16 * p + 4 * r + lk) * ld);
                if (coh) st_coh_s(C, ci, o[r]);
                else st_s(C, ci, o[r]);
            }
        }
        if (ftr) sched_signal(sc, ftr, ticket);   // waits for the stores, then a barrier
        else __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acur[t][kk] = anext[t][kk];
        cn = cnext;
    }
    return true;
}

// ---------------------------------------------------------------------------
// The factorization of one tile column J as one persistent launch: POTRF of
// the diagonal tile, the panel TRSM of every 16-row block below it and the
// trailing update of every 64 x 64 target block, run concurrently and
// pipelined on the 16-column panels of L_JJ through device counters.
// ---------------------------------------------------------------------------

// Per tile column counters (ints, zeroed once per factorization): the ticket
// counter, the number of panels of L_JJ announced by POTRF, then per 16-row
// block of the TRSM the number of its finished steps.
#define CF_TICKET 0
#define CF_PO 1
#define CF_TR 4
__host__ __device__ inline int col_tr_blocks(const Lay& L, int64_t J) { return L.s(J) * (L.b / 16) + L.ap / 16; }
__host__ __device__ inline int col_stride(const Lay& L) { return CF_TR + L.bt * (L.b / 16) + L.ap / 16; }

// Trailing-update target blocks of tile column J, 64 x 64, in this order:
//   band (J+d, J+e), 1 <= e <= d <= s:  -= L_{J+d,J} L_{J+e,J}^T   (lower blocks when d == e)
//   arrow (A, J+e):                      -= L_{A,J} L_{J+e,J}^T
//   corner (lower blocks):               -= L_{A,J} L_{A,J}^T
// (the block of (J+1, J+1) that the next POTRF needs first comes first).
struct UpBlock {
    const double* A;   // operand rows (64-row block), leading dimension lda, rows_a valid in its tile
    const double* B;
    double* O;         // target block, leading dimension ldo
    int lda, ldb, ldo;
    int rows_a, rows_b;   // valid rows from the block's first row on (<= 64)
    int ga, gb;           // TRSM row blocks (16 rows) of the first rows of A and B
    int diag;             // a diagonal block of a symmetric target: lower part only
    int* cnt;             // single-launch factor: updates applied to the target so far (else nullptr)
    int before;           // ... and how many come before this one
};

// Single-launch factor: per 64 x 64 target block, the number of tile columns
// whose update of it is done.  Band tile (K+d, K), block (i, j); arrow tile
// K, block (i, j); corner block (i, j).  Tile (I, K) of the band is updated
// by the columns max(0, I - B) .. K - 1, arrow tile K by max(0, K - B) ..
// K - 1, the corner by every column.
__host__ __device__ inline int64_t upd_band(const Lay& L, int64_t K, int d, int i, int j) {
    const int C64 = L.b / 64;
    return ((K * (L.bt + 1) + d) * C64 + i) * C64 + j;
}
__host__ __device__ inline int64_t upd_arrow(const Lay& L, int64_t K, int i, int j) {
    const int C64 = L.b / 64, na = (L.ap + 63) / 64;
    return L.nt * (int64_t)(L.bt + 1) * C64 * C64 + (K * na + i) * C64 + j;
}
__host__ __device__ inline int64_t upd_corner(const Lay& L, int i, int j) {
    const int C64 = L.b / 64, na = (L.ap + 63) / 64;
    return L.nt * (int64_t)(L.bt + 1) * C64 * C64 + L.nt * (int64_t)na * C64 + (int64_t)i * na + j;
}
__host__ __device__ inline int64_t upd_ints(const Lay& L) {
    const int na = (L.ap + 63) / 64;
    return upd_corner(L, 0, 0) + (int64_t)na * na;
}
__host__ __device__ inline int col_up_blocks(const Lay& L, int64_t J) {
    const int C64 = L.b / 64, s = L.s(J), na = (L.ap + 63) / 64;
    int cnt = 0;
    for (int d = 1; d <= s; ++d)
        for (int e = 1; e <= d; ++e) cnt += (d == e) ? C64 * (C64 + 1) / 2 : C64 * C64;
    if (L.ap > 0) cnt += s * na * C64 + na * (na + 1) / 2;
    return cnt;
}
__device__ inline UpBlock col_up_decode(double* Lm, const Lay& L, int64_t J, int t, int* upd) {
    const int C64 = L.b / 64, s = L.s(J), na = (L.ap + 63) / 64, nbr = L.b / 16, b = L.b;
    UpBlock u;
    u.cnt = nullptr;
    u.before = 0;
    for (int d = 1; d <= s; ++d) {
        for (int e = 1; e <= d; ++e) {
            const int cnt = (d == e) ? C64 * (C64 + 1) / 2 : C64 * C64;
            if (t < cnt) {
                int i, j;
                if (d == e) tri_decode(t, i, j);
                else { i = t % C64; j = t / C64; }
                u.A = Lm + L.band(J, d) + 64 * i; u.lda = b; u.rows_a = 64; u.ga = (d - 1) * nbr + 4 * i;
                u.B = Lm + L.band(J, e) + 64 * j; u.ldb = b; u.rows_b = 64; u.gb = (e - 1) * nbr + 4 * j;
                u.O = Lm + L.band(J + e, d - e) + 64 * i + (int64_t)64 * j * b; u.ldo = b;
                u.diag = (d == e && i == j);
                if (upd) {
                    u.cnt = upd + upd_band(L, J + e, d - e, i, j);
                    u.before = (int)(J - imax64(0, J + d - L.bt));
                }
                return u;
            }
            t -= cnt;
        }
    }
    const int ga0 = s * nbr;
    if (t < s * na * C64) {
        const int e = 1 + t / (na * C64), r = t % (na * C64), i = r % na, j = r / na;
        u.A = Lm + L.arrow(J) + 64 * i; u.lda = L.ap; u.rows_a = imin_(64, L.ap - 64 * i); u.ga = ga0 + 4 * i;
        u.B = Lm + L.band(J, e) + 64 * j; u.ldb = b; u.rows_b = 64; u.gb = (e - 1) * nbr + 4 * j;
        u.O = Lm + L.arrow(J + e) + 64 * i + (int64_t)64 * j * L.ap; u.ldo = L.ap;
        u.diag = 0;
        if (upd) {
            u.cnt = upd + upd_arrow(L, J + e, i, j);
            u.before = (int)(J - imax64(0, J + e - L.bt));
        }
        return u;
    }
    t -= s * na * C64;
    int i, j;
    tri_decode(t, i, j);
    u.A = Lm + L.arrow(J) + 64 * i; u.lda = L.ap; u.rows_a = imin_(64, L.ap - 64 * i); u.ga = ga0 + 4 * i;
    u.B = Lm + L.arrow(J) + 64 * j; u.ldb = L.ap; u.rows_b = imin_(64, L.ap - 64 * j); u.gb = ga0 + 4 * j;
    u.O = Lm + L.corner() + 64 * i + (int64_t)64 * j * L.ap; u.ldo = L.ap;
    u.diag = (i == j);
    if (upd) {
        u.cnt = upd + upd_corner(L, i, j);
        u.before = (int)J;
    }
    return u;
}

// Thread 0 waits until every flag[k], k < n, is at least target; then the
// workgroup goes on (false: stop, the kernel is being abandoned).
__device__ inline bool col_wait(const Sched& sc, const int* flag, int n, int target, int* sh) {
    if (threadIdx.x == 0) {
        int ok = 1;
        const int64_t t0 = wall_clock64();
        for (int k = 0; k < n && ok; ++k) {
            while (ld_coh_i(flag + k) < target) {
                if (ld_coh_i(sc.err) != 0) { ok = 0; break; }
                if (wall_clock64() - t0 > sc.spin_limit) {
                    set_error_once(sc.err, STILES_ETIMEOUT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        *sh = ok;
    }
    __syncthreads();
    const bool ok = __builtin_amdgcn_readfirstlane(*sh) != 0;
    __syncthreads();
    return ok;
}

// One 64 x 64 target block, accumulated one 16-column panel of tile column J
// at a time as the TRSM steps of its rows are announced.  Wavefront w < 4
// owns the 32 x 32 quarter (w/2, w%2), four 16 x 16 tiles; tiles past the
// valid rows, and tiles above the diagonal of a diagonal block, are not
// stored (a fifth wavefront's quarter lies past the block: it stores nothing).
__device__ inline bool col_update(const UpBlock& u, const int* ftr, int np, const Sched& sc, int* sh, int ticket) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int qi = w >> 1, qj = w & 1;
    const double* A = uniform_ptr(u.A);
    const double* B = uniform_ptr(u.B);
    double* O = (double*)uniform_ptr(u.O);
    const int ta = (u.rows_a + 15) / 16, tb = (u.rows_b + 15) / 16;   // valid 16-row tiles
    int ra[2], rb[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        ra[x] = imin_(2 * qi + x, ta - 1);
        rb[x] = imin_(2 * qj + x, tb - 1);
    }
    dbl4 acc[2][2];
    double ov[2][2][4];
    // the target as the earlier tile columns left it (device-coherent: in the
    // single-launch factor they are other workgroups of the same kernel)
    if (u.cnt && u.before > 0 && !sched_wait(sc, u.cnt, u.before, sh)) return false;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r)
                ov[x][y][r] = ld_coh_s(O, (uint32_t)((16 * ra[x] + li) + (16 * rb[y] + 4 * r + lk) * u.ldo));
        }
    // the operands of panel p + 1 are loaded (once its TRSM steps are
    // announced) while panel p is multiplied
    double av[2][4], bv[2][4], an[2][4], bn[2][4];
    auto load = [&](double (&a)[2][4], double (&b)[2][4], int p) {
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                a[x][kk] = ld_coh_s(A, (uint32_t)((16 * ra[x] + li) + (16 * p + 4 * kk + lk) * u.lda));
                b[x][kk] = ld_coh_s(B, (uint32_t)((16 * rb[x] + li) + (16 * p + 4 * kk + lk) * u.ldb));
            }
    };
    if (!col_wait(sc, ftr + u.ga, ta, 1, sh)) return false;
    if (!col_wait(sc, ftr + u.gb, tb, 1, sh)) return false;
    load(av, bv, 0);
    for (int p = 0; p < np; ++p) {
        if (p + 1 < np) {
            if (!col_wait(sc, ftr + u.ga, ta, p + 2, sh)) return false;
            if (!col_wait(sc, ftr + u.gb, tb, p + 2, sh)) return false;
            load(an, bn, p + 1);
        }
        // element r of acc[x][y]: sum_k A[16 ra + li][k] B[16 rb + 4r + lk][k]
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[y][kk], av[x][kk], acc[x][y], 0, 0, 0);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                av[x][kk] = an[x][kk];
                bv[x][kk] = bn[x][kk];
            }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int ti = 2 * qi + x, tj = 2 * qj + y;
            if (ti < ta && tj < tb && !(u.diag && ti < tj)) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    st_coh_s(O, (uint32_t)((16 * ti + li) + (16 * tj + 4 * r + lk) * u.ldo), ov[x][y][r] - acc[x][y][r]);
            }
        }
    if (u.cnt) sched_signal(sc, u.cnt, ticket);   // waits for the stores, then a barrier
    return true;
}

// Tickets, in an order where every task waits only for smaller ones (so the
// launch cannot deadlock, however many workgroups are resident): 0 is the
// POTRF of L_JJ, then the TRSM row blocks (tile J+1 first), then the update
// blocks.  The factorization of the next tile column is the next launch.
template <int NPOOL>
union ColSmemT {
    P3SmemT<NPOOL> po;
    TrSmem tr;
};
using ColSmem = ColSmemT<P3_POOL>;
// Task t of tile column J; false when the kernel must stop (a wait failed).
// upd (single-launch factor, else nullptr): the POTRF waits until the
// earlier columns' updates of its tile are in, a TRSM block until those of
// its rows are; the update blocks wait for the earlier updates of their
// targets (col_update).  gt: the task's ticket in the launch (the test hook
// Sched::withhold names one whose signals are never sent).
template <int NPOOL>
__device__ inline bool col_task(ColSmemT<NPOOL>& sm, int& sh, double* Lm, const Lay& L, int64_t J, double* Yd, int* cf,
                                const Sched& st, double* ldp, int* info, int t, int* upd, int gt) {
    const int ntr = col_tr_blocks(L, J);
    const int nbr = L.b / 16, s = L.s(J), C64 = L.b / 64;
    int* fpo = cf + CF_PO;
    int* ftr = cf + CF_TR;
    {
        TRACE(gt, 3, (unsigned long long)(t == 0 ? 0 : (t <= ntr ? 1 : 2)) | ((unsigned long long)J << 8) |
                         ((unsigned long long)t << 40));
        if (t == 0) {
            if (upd) {
                const int need = (int)(J - imax64(0, J - L.bt));
                for (int i = 0; i < C64 && need > 0; ++i)
                    if (!col_wait(st, upd + upd_band(L, J, 0, i, 0), i + 1, need, &sh)) return false;
            }
            TRACE(gt, 1, wall_clock64());
            int fail;
            double ls, lc;
            potrf3(Lm + L.band(J, 0), L.b, L.b, Yd, sm.po, &fail, &ls, &lc, gt == st.withhold ? nullptr : fpo);
            if (threadIdx.x == 0) {
                ldp[0] = ls;
                ldp[1] = lc;
                if (fail >= 0) atomicMin(info, (int)(J * L.b + fail + 1));
            }
        } else if (t <= ntr) {
            const int g = t - 1;
            double* C;
            int ld;
            if (g < s * nbr) { C = Lm + L.band(J, 1 + g / nbr) + (g % nbr) * 16; ld = L.b; }
            else { C = Lm + L.arrow(J) + (g - s * nbr) * 16; ld = L.ap; }
            if (upd) {
                bool ok = true;
                if (g < s * nbr) {
                    const int d = 1 + g / nbr;
                    const int need = (int)(J - imax64(0, J + d - L.bt));
                    if (need > 0) ok = col_wait(st, upd + upd_band(L, J, d, (g % nbr) / 4, 0), C64, need, &sh);
                } else {
                    const int need = (int)(J - imax64(0, J - L.bt));
                    if (need > 0) ok = col_wait(st, upd + upd_arrow(L, J, (g - s * nbr) / 4, 0), C64, need, &sh);
                }
                if (!ok) return false;
            }
            TRACE(gt, 1, wall_clock64());
            if (!tr_panel(C, ld, Lm + L.band(J, 0), Yd, L.b, fpo, ftr + g, st, sm.tr, gt)) return false;
        } else {
            const UpBlock u = col_up_decode(Lm, L, J, t - 1 - ntr, upd);
            TRACE(gt, 1, wall_clock64());
            if (!col_update(u, ftr, L.b / 16, st, &sh, gt)) return false;
        }
    }
    TRACE(gt, 2, wall_clock64());
    return true;
}
// The whole factor of the band tile columns in one persistent launch.
// Ticket g is task g - off[J] of tile column J (off: first ticket of each
// column, off[N] = all), so the tasks go column by column and, inside a
// column, in the order above: every wait is for a smaller ticket, and the
// launch cannot deadlock however many workgroups are resident.  Across
// columns the tasks wait on the update counters (col_task): the POTRF of
// column J+1 starts as soon as column J's updates of its tile are in, while
// the rest of column J's trailing update goes on.
__global__ __launch_bounds__(P3_NT) void k_factor_all(double* Lm, Lay L, double* Yd, int* cf, int* upd, const int* off,
                                                   Sched sc, double* ldp, int* info) {
    __shared__ ColSmem sm;
    __shared__ int sh;
    const int64_t N = L.nt;
    const int ntot = off[N];
    const int cstride = col_stride(L);
    for (;;) {
        const int g = sched_next(sc, ntot, &sh);
        if (g < 0) return;
        TRACE(g, 0, wall_clock64());
        int lo = 0, hi = (int)N;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (off[mid] <= g) lo = mid; else hi = mid;
        }
        const int64_t J = lo;
        if (!col_task(sm, sh, Lm, L, J, Yd + J * (int64_t)L.b * 16, cf + J * cstride, sc, ldp + 2 * J, info,
                      g - off[J], upd, g))
            return;
    }
}

// First ticket of every tile column (off[N] = all tickets), and the ticket counter.
// A column's task count depends on J only through s(J): every column before
// J1 = N - B has the full count, so off[J] is J1 (or J) times that count plus
// at most B tail terms, one thread per entry.
__global__ void k_factor_offsets(Lay L, int* off, int* ticket) {
    const int64_t N = L.nt, J1 = imax64(0, N - L.bt);
    const int64_t cs = J1 > 0 ? 1 + col_tr_blocks(L, 0) + col_up_blocks(L, 0) : 0;
    for (int64_t J = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; J <= N; J += (int64_t)gridDim.x * blockDim.x) {
        int64_t acc = (J < J1 ? J : J1) * cs;
        for (int64_t K = J1; K < J; ++K) acc += 1 + col_tr_blocks(L, K) + col_up_blocks(L, K);
        off[J] = (int)acc;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;
}

// C (rows x rows, lower blocks) -= P P^T, P rows x K (generic, corner blocking).
__global__ __launch_bounds__(NT) void k_syrk_generic(double* C, int64_t ldc, const double* P,
                                                    int64_t ldp, int rows, int K) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    int rb, cb;
    tri_decode(blockIdx.x, rb, cb);
    const int va = imin_(64, rows - rb * 64), vb = imin_(64, rows - cb * 64);
    GAcc g;
    gacc_zero(g);
    gemm_acc(g, opnd(P + rb * 64, ldp, 0, va), opnd(P + cb * 64, ldp, 1, vb), K, smem);
    double* O = C + rb * 64 + (int64_t)cb * 64 * ldc;
    gemm_store(g, smem, -1.0, 1.0, O, ldc, O, ldc, va, vb);
}

__global__ void k_zero_block(double* C, int64_t ld, int rows, int cols) {
    for (int idx = threadIdx.x + blockIdx.x * blockDim.x; idx < rows * cols; idx += blockDim.x * gridDim.x)
        C[(idx % rows) + (int64_t)(idx / rows) * ld] = 0.0;
}

// Final log det (Neumaier sum of the per-block partials, in order) and info.
__device__ inline void factor_final_body(const double* ldp, int nparts, const int* info_ws, const int* err,
                                         double* logdet, int* info) {
    double s = 0.0, c = 0.0;
    for (int i = 0; i < nparts; ++i) {
        neumaier(s, c, ldp[2 * i]);
        neumaier(s, c, ldp[2 * i + 1]);
    }
    const int f = (*err != 0) ? *err : *info_ws;
    *info = (f == 0x7fffffff) ? 0 : f;
    *logdet = (f == 0x7fffffff) ? (s + c) : __builtin_nan("");
}
__global__ void k_factor_final(const double* ldp, int nparts, const int* info_ws, const int* err, double* logdet,
                               int* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    factor_final_body(ldp, nparts, info_ws, err, logdet, info);
}

// ---------------------------------------------------------------------------
// Selected-inversion kernels
// ---------------------------------------------------------------------------

// Phase 1, diagonal tiles: X_J = L_JJ^{-1} ("TRSM(L_ii^T, I)"), stored in the
// diagonal slots of the workspace; the corner inverse likewise.
__device__ inline void trtri_body(const double* Lm, double* W, const Lay& L, int* info, int bid, double* smem) {
    const int64_t J = bid;
    int bad;
    if (J < L.nt) {
        trtri_tile(Lm + L.band(J, 0), L.b, W + L.band(J, 0), L.b, L.b, smem, &bad);
    } else {
        trtri_tile(Lm + L.corner(), L.ap, W + L.corner(), L.ap, L.ap, smem, &bad);
    }
    if (threadIdx.x == 0 && bad) atomicExch(info, STILES_EBADL);
}
// (j0: first tile column; the launches of a selection start there)
__global__ __launch_bounds__(NT) void k_trtri_all(const double* Lm, double* W, Lay L, int* info, int64_t j0) {
    __shared__ double smem[TRTRI_SMEM_DOUBLES];
    trtri_body(Lm, W, L, info, (int)(blockIdx.x + j0), smem);
}

// Rows of the panel below tile J (band tiles J+1..J+s, then the arrow tile),
// 64-row block blk.
__device__ inline void panel_rows(const Lay& L, double* base, int64_t J, int blk, double*& C,
                                  int64_t& ld, int& valid) {
    const int nb64 = L.b / 64;
    const int s = L.s(J);
    if (blk < s * nb64) {
        const int d = 1 + blk / nb64, rb = blk % nb64;
        C = base + L.band(J, d) + rb * 64;
        ld = L.b;
        valid = 64;
    } else {
        const int rb = blk - s * nb64;
        C = base + L.arrow(J) + rb * 64;
        ld = L.ap;
        valid = imin_(64, L.ap - rb * 64);
    }
}

// Phase 1, off-diagonal tiles: Lhat_{k,J} = L_{k,J} X_J for the band tiles
// k = J+1..J+s and the arrow tile ("TRMM").  Grid: (J, 64-row block, col block).
__device__ inline void trmm_body(const double* Lm, double* W, const Lay& L, int bid, double* smem) {
    const int nb64 = L.b / 64;
    const int nab = arrow_blocks(L.ap);
    const int rows_max = L.bt * nb64 + nab;
    const int64_t J = bid / (rows_max * nb64);
    const int r = (int)(bid % (rows_max * nb64));
    const int blk = r / nb64, cb = r % nb64;
    const int s = L.s(J);
    if (blk >= s * nb64 + nab) return;
    double* Cw;
    int64_t ld;
    int valid;
    panel_rows(L, W, J, blk, Cw, ld, valid);
    const double* Cl = Lm + (Cw - W);
    const double* X = W + L.band(J, 0);
    const int k0 = cb * 64;
    GAcc g;
    gacc_zero(g);
    gemm_acc(g, opnd(Cl + (int64_t)k0 * ld, ld, 0, valid), opnd(X + k0 + (int64_t)k0 * L.b, L.b, 0, 64),
             L.b - k0, smem);
    gemm_store(g, smem, 1.0, 0.0, nullptr, 0, Cw + (int64_t)k0 * ld, ld, valid, 64);
}
__global__ __launch_bounds__(NT) void k_trmm_all(const double* Lm, double* W, Lay L, int64_t j0) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    const int nb64 = L.b / 64;
    trmm_body(Lm, W, L, xcd_block((int)blockIdx.x, (int)gridDim.x) + (int)(j0 * (L.bt * nb64 + arrow_blocks(L.ap)) * nb64),
              smem);
}

// Phase 2 initial value of each diagonal tile, "LAUUM": Sigma_JJ = X_J^T X_J
// (and the corner Sigma_AA = X_A^T X_A, which is final).  Lower 64 x 64
// blocks, mirrored so the tiles are full symmetric.  Blocks are numbered
// densely: lauum_per(L) per band tile column, then the corner's
// (lauum_corner(L), none without an arrow).
__host__ __device__ inline int lauum_per(const Lay& L) {
    const int nb64 = L.b / 64;
    return nb64 * (nb64 + 1) / 2;
}
__host__ __device__ inline int lauum_corner(const Lay& L) {
    const int nab = arrow_blocks(L.ap);
    return L.ap > 0 ? nab * (nab + 1) / 2 : 0;
}
// blocks of tile columns j0.. and the corner
__host__ __device__ inline int64_t lauum_blocks(const Lay& L, int64_t j0) {
    return (L.nt - j0) * (int64_t)lauum_per(L) + lauum_corner(L);
}
__device__ inline void lauum_body(const double* W, double* S, const Lay& L, int64_t bid, double* smem) {
    const int per = lauum_per(L);
    const int64_t nband = L.nt * (int64_t)per;
    const double* X;
    double* O;
    int m;
    int64_t ld;
    int t;
    if (bid < nband) {
        const int64_t J = bid / per;
        t = (int)(bid % per);
        X = W + L.band(J, 0); O = S + L.band(J, 0); m = L.b; ld = L.b;
    } else {
        t = (int)(bid - nband);
        if (t >= lauum_corner(L)) return;
        X = W + L.corner(); O = S + L.corner(); m = L.ap; ld = L.ap;
    }
    int rb, cb;
    tri_decode(t, rb, cb);
    const int k0 = rb * 64;
    const int va = imin_(64, m - rb * 64), vb = imin_(64, m - cb * 64);
    GAcc g;
    gacc_zero(g);
    gemm_acc(g, opnd(X + k0 + (int64_t)rb * 64 * ld, ld, 1, va), opnd(X + k0 + (int64_t)cb * 64 * ld, ld, 0, vb),
             m - k0, smem);
    gemm_store_sym(g, smem, 1.0, 0.0, nullptr, 0, O + rb * 64 + (int64_t)cb * 64 * ld,
                   O + cb * 64 + (int64_t)rb * 64 * ld, ld, rb == cb, va, vb);
}
__global__ __launch_bounds__(NT) void k_lauum_all(const double* W, double* S, Lay L, int64_t j0) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    lauum_body(W, S, L, xcd_block((int)blockIdx.x, (int)gridDim.x) + j0 * lauum_per(L), smem);
}

#define ARW (-1)   // "the arrow" in place of a band tile offset

// ---------------------------------------------------------------------------
// Phase 2 as one persistent kernel
// ---------------------------------------------------------------------------
// Tile column J needs the off-diagonal tiles S(J) x S(J) of Sigma, where
// S(J) = band tiles J+1..J+s and the arrow.  Each output block is summed over
// k in three parts, by how late its operands become final:
//   k over the far tiles J+3..J+s and the arrow: final once the off-diagonal
//     tiles of column J+2 are (two and a half columns ahead);
//   k = J+2: final once column J+2 is done;
//   k = J+1: final once column J+1's off-diagonal tiles (rows i far) or its
//     diagonal tile (row J+1) are.
// With two parts (Lay::p2s == 2) the k = J+2 term stays in the far parts:
// EA and E1A sum over k = J+2.., EB and E1B have no tasks, EA(J) waits for
// done(J+2) and E1A(J) for L1(J+1) and far(J+1), L and L1 read the partial of
// EA and E1A, and the group order is [EA(G-1), L(G), L1(G), E1A(G-1), DA(G),
// DB(G)].
// Every task is a 32 x 32 block whose reduction is spread over the 4
// wavefronts of a workgroup, so that the tasks on the dependency chain stay
// short ("far rows" = tiles J+2..J+s and the arrow):
//   EA : Sigma_{i,J}   = -sum_{k = J+3.., arrow} Sigma_{i,k} Lhat_{k,J}   i far
//   EB : Sigma_{i,J}  -= Sigma_{i,J+2} Lhat_{J+2,J}                      i far
//   L  : Sigma_{i,J}  -= Sigma_{i,J+1} Lhat_{J+1,J}                      i far
//   E1A: Sigma_{J+1,J} = -sum_{k = J+3.., arrow} Sigma_{J+1,k} Lhat_{k,J}
//   E1B: Sigma_{J+1,J} -= Sigma_{J+1,J+2} Lhat_{J+2,J}
//   L1 : Sigma_{J+1,J} -= Sigma_{J+1,J+1} Lhat_{J+1,J}
//   DA : Sigma_JJ = X_J^T X_J - sum_{i far} Lhat_{i,J}^T Sigma_{i,J}       (lower blocks)
//   DB : Sigma_JJ -= Lhat_{J+1,J}^T Sigma_{J+1,J}, then mirrored           (lower blocks)
// Dependencies (counters per kind and tile column; "offdiag(J)": L(J), L1(J)
// done, or EA(J) for the last column; "far(J)": L(J) done, or EA(J) for the
// last column; "done(J)": DB(J), or DA(J) for the last column):
//   EA(J): offdiag(J+2);          EB(J): done(J+2), EA(J);
//   E1A(J): far(J+1);             E1B(J): L1(J+1), E1A(J);
//   L(J): offdiag(J+1), EB(J) (EA(J) when s < 2);
//   L1(J): done(J+1), E1B(J) (E1A(J) when s < 2);
//   DA(J): far(J);                DB(J): DA(J), L1(J).
// Ticket order: groups G = N-1 .. 0, group G = [EA(G-1), L(G), E1B(G),
// E1A(G-1), EB(G-1), L1(G), DA(G), DB(G)] (group N-1 also starts with
// EA(N-1)); every task depends only on tasks of earlier groups or earlier in
// its own group.  The order puts each task's ticket close to the time it
// becomes ready, so few workgroups sit on a ticket that is still waiting (it
// was the fastest of the orders timed).
enum { P2_EA = 0, P2_EB, P2_E1A, P2_E1B, P2_L, P2_L1, P2_DA, P2_DB, P2_KINDS };

struct P2 {
    double* S;
    const double* W;
    Lay L;
    int* cnt;        // [P2_KINDS * N] finished tasks per kind and tile column
    int ntasks;
    // groups are taken in the order G = N-1-q, q = 0, 1, ...; from q = q0 on,
    // every group but the last (G = 0) holds g_tasks tasks, and group q0
    // starts at ticket off_q0, so a ticket's group is found in closed form
    int q0, off_q0, g_tasks;
};

struct P2Counts {
    int n[P2_KINDS];
};

// Task counts of tile column J.  EA and E1A exist (possibly with an empty
// reduction, writing zeros) wherever their rows do.
__host__ __device__ inline P2Counts p2_counts(const Lay& L, int64_t J) {
    P2Counts c;
    const int s = L.s(J);
    const int C32 = L.b / 32;
    const int far = s > 1 ? s - 1 : 0;
    const int nf32 = far * C32 + (L.ap + 31) / 32;
    const bool three = L.p2s == 3;
    c.n[P2_EA] = nf32 * C32;
    c.n[P2_EB] = three && s >= 2 ? nf32 * C32 : 0;
    c.n[P2_E1A] = s >= 1 ? C32 * C32 : 0;
    c.n[P2_E1B] = three && s >= 2 ? C32 * C32 : 0;
    c.n[P2_L] = s >= 1 ? nf32 * C32 : 0;
    c.n[P2_L1] = s >= 1 ? C32 * C32 : 0;
    c.n[P2_DA] = C32 * (C32 + 1) / 2;
    c.n[P2_DB] = s >= 1 ? C32 * (C32 + 1) / 2 : 0;
    return c;
}

// Task count of one kind (a switch rather than indexing P2Counts::n with a
// run-time kind, which would put the array in scratch memory).
__host__ __device__ inline int p2_count(const Lay& L, int64_t J, int kind) {
    const P2Counts c = p2_counts(L, J);
    switch (kind) {
        case P2_EA: return c.n[P2_EA];
        case P2_EB: return c.n[P2_EB];
        case P2_E1A: return c.n[P2_E1A];
        case P2_E1B: return c.n[P2_E1B];
        case P2_L: return c.n[P2_L];
        case P2_L1: return c.n[P2_L1];
        case P2_DA: return c.n[P2_DA];
        default: return c.n[P2_DB];
    }
}

// Slot i of group G: the kind and the tile column offset (0 or -1) of its
// tasks (with two parts, EB and E1B come last and have no tasks).
#define P2_SLOTS 8
// (a switch, not tables: a table indexed at run time would live in scratch
// memory)
__host__ __device__ inline void p2_slot(const Lay& L, int i, int& kind, int& dj) {
    if (L.p2s == 3) {
        switch (i) {
            case 0: kind = P2_EA; dj = -1; break;
            case 1: kind = P2_L; dj = 0; break;
            case 2: kind = P2_E1B; dj = 0; break;
            case 3: kind = P2_E1A; dj = -1; break;
            case 4: kind = P2_EB; dj = -1; break;
            case 5: kind = P2_L1; dj = 0; break;
            case 6: kind = P2_DA; dj = 0; break;
            default: kind = P2_DB; dj = 0;
        }
    } else {
        switch (i) {
            case 0: kind = P2_EA; dj = -1; break;
            case 1: kind = P2_L; dj = 0; break;
            case 2: kind = P2_L1; dj = 0; break;
            case 3: kind = P2_E1A; dj = -1; break;
            case 4: kind = P2_DA; dj = 0; break;
            case 5: kind = P2_DB; dj = 0; break;
            case 6: kind = P2_EB; dj = -1; break;
            default: kind = P2_E1B; dj = 0;
        }
    }
}

// Tasks in group G (see the ticket order above).
__host__ __device__ inline int p2_group_tasks(const Lay& L, int64_t G) {
    const P2Counts c = p2_counts(L, G);
    int t = (G == L.nt - 1) ? c.n[P2_EA] : 0;
    if (G >= 1) {
        const P2Counts c1 = p2_counts(L, G - 1);
        t += c1.n[P2_EA] + c1.n[P2_E1A] + c1.n[P2_EB];
    }
    return t + c.n[P2_E1B] + c.n[P2_L] + c.n[P2_L1] + c.n[P2_DA] + c.n[P2_DB];
}

__device__ inline void p2_setup_body(const P2& p, int* ticket, int* err) {
    const Lay& L = p.L;
    for (int64_t i = threadIdx.x; i < P2_KINDS * L.nt; i += blockDim.x) p.cnt[i] = 0;
    if (threadIdx.x == 0) {
        *ticket = 0;
        *err = 0;
    }
}
__global__ void k_p2_setup(P2 p, int* ticket, int* err) { p2_setup_body(p, ticket, err); }

// Operand A = Sigma restricted to a block of rows and a tile of k:
// rows = block rbl (of rb rows) of tile J+d (d >= 1) or of the arrow (ARW);
// k = tile J+e (e >= 1) or the arrow.
__device__ inline void p2_sigma_rows(const Lay& L, const double* S, int64_t J, int d, int rbl, int rb, int e,
                                     const double*& a, int64_t& lda, int& ta, int& av) {
    av = rb;
    if (d != ARW && e != ARW) {
        if (d > e) { a = S + L.band(J + e, d - e) + rbl * rb; lda = L.b; ta = 0; }
        else if (d == e) { a = S + L.band(J + d, 0) + rbl * rb; lda = L.b; ta = 0; }
        else { a = S + L.band(J + d, e - d) + (int64_t)rbl * rb * L.b; lda = L.b; ta = 1; }
    } else if (d != ARW) {
        a = S + L.arrow(J + d) + (int64_t)rbl * rb * L.ap; lda = L.ap; ta = 1;
    } else {
        av = imin_(rb, L.ap - rbl * rb);
        lda = L.ap; ta = 0;
        a = (e != ARW) ? S + L.arrow(J + e) + rbl * rb : S + L.corner() + rbl * rb;
    }
}

// Row block rbg (of rb rows) among the far rows of S(J): tiles J+2..J+s, arrow.
__device__ inline void p2_far_row(const Lay& L, int s, int rbg, int rb, int& d, int& rbl) {
    const int per = L.b / rb;
    const int far = s > 1 ? s - 1 : 0;
    if (rbg < far * per) { d = 2 + rbg / per; rbl = rbg % per; }
    else { d = ARW; rbl = rbg - far * per; }
}

// Every task of the given kind and tile column finished (nothing to wait for
// past the last column).
__device__ inline void p2_dep_all(const P2& p, SchedDeps& d, int kind, int64_t J) {
    if (J < p.L.nt) deps_add(d, &p.cnt[kind * p.L.nt + J], p2_count(p.L, J, kind));
}
// done(J): all of column J final.
__device__ inline void p2_dep_done(const P2& p, SchedDeps& d, int64_t J) {
    if (J < p.L.nt) p2_dep_all(p, d, p.L.s(J) >= 1 ? P2_DB : P2_DA, J);
}
// far(J): the far rows of column J final.
__device__ inline void p2_dep_far(const P2& p, SchedDeps& d, int64_t J) {
    if (J < p.L.nt) p2_dep_all(p, d, p.L.s(J) >= 1 ? P2_L : P2_EA, J);
}
// offdiag(J): every off-diagonal tile of column J final.
__device__ inline void p2_dep_offdiag(const P2& p, SchedDeps& d, int64_t J) {
    if (J >= p.L.nt) return;
    if (p.L.s(J) >= 1) {
        p2_dep_all(p, d, P2_L, J);
        p2_dep_all(p, d, P2_L1, J);
    } else {
        p2_dep_all(p, d, P2_EA, J);
    }
}

// LDS of a Phase 2 workgroup: the wavefronts' staging areas, which
// wave_reduce reuses for the partial blocks (the larger of the two), then the
// reduced block.  Both kernels run two workgroups per CU.  The single-matrix
// kernel stages 16-deep chunks; the batched one 8-deep chunks, which halve its
// LDS (41 against 72 KB), so that the kernels of other serving lanes still
// find room on a CU beside it.  (Three batched workgroups per CU, which the
// 8-deep chunks allow, made a batched pass faster alone, 125 against 141 ms,
// but filled every CU: concurrent serving lanes then lost capacity, and in the
// 2,000-job served stream one batch's selected inverse hit the wait limit.)
template <int KC>
struct P2Cfg {
    static constexpr int STAGE = WS<KC>::SMEM > WR_SMEM_DOUBLES ? WS<KC>::SMEM : WR_SMEM_DOUBLES;
    static constexpr int SMEM = STAGE + 32 * WR_LD;
    static constexpr int WG_PER_CU = 2;
};
#define P2_KC_SINGLE 16
#define P2_KC_BATCHED 8

// One Phase 2 task: a 32 x 32 output block, its reduction spread over the 4
// wavefronts.
template <int KC>
__device__ __forceinline__ void p2_task_small(const P2& p, int kind, int64_t J, int u, bool mirror_da, double* smem,
                                           double* red, int t) {
    const Lay& L = p.L;
    const int C32 = L.b / 32;
    const int s = L.s(J);
    const int far = s > 1 ? s - 1 : 0;
    // the reduction: band tiles J+e0 .. J+e0+nband-1, then the arrow if karw
    int e0, nband;
    bool karw;
    const int ef = L.p2s == 3 ? 3 : 2;   // first band tile of the far parts
    switch (kind) {
        case P2_EA: case P2_E1A: e0 = ef; nband = s >= ef ? s - ef + 1 : 0; karw = L.ap > 0; break;
        case P2_EB: case P2_E1B: e0 = 2; nband = 1; karw = false; break;
        case P2_DA: e0 = 2; nband = far; karw = L.ap > 0; break;
        default: e0 = 1; nband = 1; karw = false;   // L, L1, DB
    }
    const int nseg = nband + (karw ? 1 : 0);
    const int ktot = nband * L.b + (karw ? L.ap : 0);
    // the output block
    int d = 0, rbl = 0, rb = 0, cb = 0;
    const bool rowtask = kind < P2_DA;
    if (rowtask) {
        if (kind == P2_EA || kind == P2_EB || kind == P2_L) p2_far_row(L, s, u / C32, 32, d, rbl);
        else { d = 1; rbl = u / C32; }
        cb = u % C32;
    } else {
        tri_decode(u, rb, cb);
    }
    const bool zero_base = kind == P2_EA || kind == P2_E1A;
    double* O;
    int64_t ldo;
    int mv = 32;
    if (rowtask) {
        if (d != ARW) { O = p.S + L.band(J, d) + rbl * 32 + (int64_t)cb * 32 * L.b; ldo = L.b; }
        else { O = p.S + L.arrow(J) + rbl * 32 + (int64_t)cb * 32 * L.ap; ldo = L.ap; mv = imin_(32, L.ap - rbl * 32); }
    } else {
        O = p.S + L.band(J, 0) + rb * 32 + (int64_t)cb * 32 * L.b;
        ldo = L.b;
    }
    const bool diag = (kind >= P2_DA) && rb == cb;
    // the partial already stored (EB, E1B, L, L1, DB) is final once the task
    // runs: read it now so its round trip overlaps the products
    // (unconditional loads from inside the block, the unused ones dropped
    // when the partial is applied: a load under a branch would make the
    // compiler wait for it before the products)
    double ov[4] = {0.0, 0.0, 0.0, 0.0};
    if (!zero_base) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q, i = imin_(e & 31, mv - 1), j = e >> 5;
            ov[q] = ld_coh(O + i + (int64_t)j * ldo);
        }
    }
    dbl4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    wave_segs<KC>(acc, nseg, ktot, smem, [&](int q) {
        const int e = (q < nband) ? e0 + q : ARW;
        if (rowtask) {
            const double* a; int64_t lda; int ta, av;
            p2_sigma_rows(L, p.S, J, d, rbl, 32, e, a, lda, ta, av);
            if (e != ARW)
                return mkseg(a, lda, ta, p.W + L.band(J, e) + (int64_t)cb * 32 * L.b, L.b, 0, L.b, av, 1, 0);
            return mkseg(a, lda, ta, p.W + L.arrow(J) + (int64_t)cb * 32 * L.ap, L.ap, 0, L.ap, av, 1, 0);
        }
        if (e != ARW)
            return mkseg(p.W + L.band(J, e) + (int64_t)rb * 32 * L.b, L.b, 1,
                         p.S + L.band(J, e) + (int64_t)cb * 32 * L.b, L.b, 0, L.b, 32, 0, 1);
        return mkseg(p.W + L.arrow(J) + (int64_t)rb * 32 * L.ap, L.ap, 1,
                     p.S + L.arrow(J) + (int64_t)cb * 32 * L.ap, L.ap, 0, L.ap, 32, 0, 1);
    });
    TRACE(t, 4, wall_clock64());
    wave_reduce(acc, smem, red);
    TRACE(t, 5, wall_clock64());
    // out = base - red, base = the partial already stored (EB, E1B, L, L1,
    // DB), Sigma_JJ's initial value X^T X (DA), or 0 (EA, E1A)
    const bool mirror = (kind == P2_DB) || (kind == P2_DA && mirror_da);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q, i = e & 31, j = e >> 5;
        if (i >= mv || (diag && i < j)) continue;
        red[j * WR_LD + i] = (zero_base ? 0.0 : ov[q]) - red[j * WR_LD + i];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int i = e & 31, j = e >> 5;
        if (i >= mv) continue;
        if (diag && i < j) {
            if (mirror) st_coh(O + i + (int64_t)j * ldo, red[i * WR_LD + j]);
            continue;
        }
        const double v = red[j * WR_LD + i];
        st_coh(O + i + (int64_t)j * ldo, v);
        if (mirror && !diag) st_coh(p.S + L.band(J, 0) + (cb * 32 + j) + (int64_t)(rb * 32 + i) * L.b, v);
    }
    TRACE(t, 6, wall_clock64());
}

template <int KC>
__device__ inline void p2_run(const P2& p, const Sched& sc, double* smem, int* sh) {
    double* red = smem + P2Cfg<KC>::STAGE;
    const Lay& L = p.L;
    const int64_t N = L.nt;
    for (;;) {
        const int t = sched_next(sc, p.ntasks, &sh[0]);
        if (t < 0) break;
        TRACE(t, 0, wall_clock64());
        // the group of ticket t: in closed form past group q0, else by
        // walking the first q0 groups (arithmetic only, no memory reads)
        int64_t q;
        int base;
        if (t >= p.off_q0) {
            q = p.q0 + (t - p.off_q0) / p.g_tasks;
            if (q > N - 1) q = N - 1;
            base = p.off_q0 + (int)(q - p.q0) * p.g_tasks;
        } else {
            q = 0;
            base = 0;
            for (;;) {
                const int n = p2_group_tasks(L, N - 1 - q);
                if (t < base + n) break;
                base += n;
                ++q;
            }
        }
        const int64_t G = N - 1 - q;       // group
        int u = t - base;
        // decode (kind, J, index) inside group G
        int kind = -1;
        int64_t J = G;
        if (G == N - 1) {
            const int n = p2_counts(L, G).n[P2_EA];
            if (u < n) kind = P2_EA;
            else u -= n;
        }
        for (int i = 0; kind < 0 && i < P2_SLOTS; ++i) {
            int k, dj;
            p2_slot(L, i, k, dj);
            if (G + dj < 0) continue;
            const int n = p2_count(L, G + dj, k);
            if (u < n) { kind = k; J = G + dj; }
            else u -= n;
        }
        int* my = &p.cnt[kind * N + J];

        // dependencies, all polled together
        SchedDeps dp;
        dp.n = 0;
        const bool three = L.p2s == 3;
        const bool two = three && L.s(J) >= 2;   // EB / E1B hold the partial
        switch (kind) {
            case P2_EA:
                if (three) p2_dep_offdiag(p, dp, J + 2);
                else p2_dep_done(p, dp, J + 2);
                break;
            case P2_EB: p2_dep_done(p, dp, J + 2); p2_dep_all(p, dp, P2_EA, J); break;
            case P2_E1A:
                if (!three) p2_dep_all(p, dp, P2_L1, J + 1);
                p2_dep_far(p, dp, J + 1);
                break;
            case P2_E1B: p2_dep_all(p, dp, P2_L1, J + 1); p2_dep_all(p, dp, P2_E1A, J); break;
            case P2_L: p2_dep_offdiag(p, dp, J + 1); p2_dep_all(p, dp, two ? P2_EB : P2_EA, J); break;
            case P2_L1: p2_dep_done(p, dp, J + 1); p2_dep_all(p, dp, two ? P2_E1B : P2_E1A, J); break;
            case P2_DA: p2_dep_far(p, dp, J); break;
            default: p2_dep_all(p, dp, P2_DA, J); p2_dep_all(p, dp, P2_L1, J);
        }
        if (!sched_wait_deps(sc, dp, &sh[1])) break;
        TRACE(t, 1, wall_clock64());

        p2_task_small<KC>(p, kind, J, u, L.s(J) == 0, smem, red, t);
        sched_signal(sc, my, t);
        TRACE(t, 2, wall_clock64());
        TRACE(t, 3, (unsigned long long)kind | ((unsigned long long)J << 8) | ((unsigned long long)blockIdx.x << 40));
        TRACE(t, 7, (unsigned long long)__smid());
    }
}
__global__ __launch_bounds__(NT) void k_phase2(P2 p, Sched sc) {
    __shared__ double smem[P2Cfg<P2_KC_SINGLE>::SMEM];
    __shared__ int sh[2];
    p2_run<P2_KC_SINGLE>(p, sc, smem, sh);
}

__global__ void k_selinv_final(const int* info_ws, const int* err, int* info) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *info = (*err != 0) ? *err : *info_ws;
}

// ---------------------------------------------------------------------------
// Batched form: many independent matrices per launch
// ---------------------------------------------------------------------------
// Every launch of the single-matrix path becomes one launch over all the
// matrices of a batch that have work in it: a table of segments maps each
// workgroup to (matrix, workgroup index within that matrix's share), and
// every matrix keeps its own tickets, counters and workspace, so the tasks,
// their decomposition and their arithmetic are those of the single-matrix
// path, matrix by matrix (results are identical bit for bit).

// Sub-buffers of a factor workspace (shared by both forms).
struct FactorWs {
    int* winfo;     // first failing column (atomicMin), 0x7fffffff when none
    int* err;       // scheduler error word
    double* ldp;    // log det partial pairs, N + 2 of them
    double* Xc;     // 256 x 256 inverse of the blocked corner
    double* Yd;     // 16 x 16 diagonal-block inverses of every L_JJ
    int* cf;        // per tile column counters
    int* upd;       // update counters of the single-launch factor (upd_ints)
    int* off;       // first ticket of every tile column (N + 1)
    int* ticket;
};
__host__ __device__ inline FactorWs factor_ws(const Lay& L, char* ws) {
    FactorWs f;
    f.winfo = (int*)ws;
    f.err = f.winfo + 16;
    f.ldp = (double*)(ws + WS_HEAD);
    f.Xc = f.ldp + 2 * (L.nt + 2);
    f.Yd = f.Xc + 256 * 256;
    f.cf = (int*)(f.Yd + L.nt * (int64_t)L.b * 16);
    f.upd = f.cf + L.nt * (int64_t)col_stride(L);
    f.off = f.upd + upd_ints(L);
    f.ticket = f.winfo + 32;
    return f;
}

// Sub-buffers of a selinv workspace.
struct SelinvWs {
    int* winfo;     // selinv info
    int* ticket;    // Phase 2 ticket counter
    int* err;       // Phase 2 scheduler error word
    double* W;      // Phase 1 tiles (tile layout)
    int* flags;     // Phase 2 ready counters
};
__host__ __device__ inline SelinvWs selinv_ws(const Lay& L, char* ws) {
    SelinvWs v;
    v.winfo = (int*)ws;
    v.ticket = v.winfo + 16;
    v.err = v.winfo + 32;
    v.W = (double*)(ws + WS_HEAD);
    v.flags = (int*)(v.W + L.total);
    return v;
}

__host__ __device__ inline P2 make_p2(double* S, const SelinvWs& v, const Lay& L, int ntasks) {
    P2 p;
    p.S = S;
    p.W = v.W;
    p.L = L;
    p.cnt = v.flags;
    p.ntasks = ntasks;
    const int64_t N = L.nt;
    const int64_t qr = L.bt > 1 ? L.bt : 1;
    p.q0 = (int)(N - 1 < qr ? N - 1 : qr);
    p.off_q0 = 0;
    for (int q = 0; q < p.q0; ++q) p.off_q0 += p2_group_tasks(L, N - 1 - q);
    p.g_tasks = p.q0 < N - 1 ? p2_group_tasks(L, N - 1 - p.q0) : 1;
    return p;
}

// One matrix of a batch, as the device sees it.
struct BInst {
    Lay L;
    const double* A;
    double* Lm;
    double* S;
    double* logdet;
    int* info;        // [0] factor, [1] selinv
    char* ws;         // this matrix's workspace (factor or selinv layout)
    int p2_tasks;     // Phase 2 task count
    int nparts;       // log det partial pairs (tile columns + corner blocks)
};
// Workgroups [first, next first) of a launch belong to matrix inst; a table
// of nseg segments ends with a sentinel holding the launch's grid size.
struct BSeg {
    int inst;
    int first;
};
struct BArgs {
    const BInst* bi;
    const BSeg* seg;
    int nseg;
    int64_t spin_limit;
};
__device__ inline int bseg_find(const BSeg* seg, int nseg, int b) {
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid].first <= b) lo = mid; else hi = mid;
    }
    return lo;
}
// the matrix of logical block B, B's index within the matrix's share, and
// the share's size
#define BATCH_DECODE_AT(a, I, bid, nblk, B)                                    \
    const int b_ = (B);                                                        \
    const int q_ = bseg_find((a).seg, (a).nseg, b_);                           \
    const BInst& I = (a).bi[(a).seg[q_].inst];                                 \
    const int bid = b_ - (a).seg[q_].first;                                    \
    const int nblk = (a).seg[q_ + 1].first - (a).seg[q_].first;                \
    (void)nblk
// ... of this workgroup.  (The XCD grouping of the single-matrix Phase 1
// products, applied to the batched ones, made them slower: kb_lauum 597 ->
// 762 us per pass; not used here.)
#define BATCH_DECODE(a, I, bid, nblk) BATCH_DECODE_AT(a, I, bid, nblk, (int)blockIdx.x)

// Factor set-up of every matrix (one workgroup per matrix): info and error
// words, tile column counters and update counters (contiguous).
__global__ __launch_bounds__(NT) void kb_factor_setup(const BInst* bi) {
    const BInst& I = bi[blockIdx.x];
    const FactorWs f = factor_ws(I.L, I.ws);
    if (threadIdx.x == 0) {
        *f.winfo = 0x7fffffff;
        *f.err = 0;
    }
    const int64_t n = I.L.nt * (int64_t)col_stride(I.L) + upd_ints(I.L);
    for (int64_t i = threadIdx.x; i < n; i += NT) f.cf[i] = 0;
}

// Tile columns J0 .. J0 + ncol - 1 of every matrix (those with N > J) in one
// launch, all their tasks on one ticket queue, column after column.  Inside
// column c, ticket tb[c] + g is local task t of matrix order[g - off[t]] (the
// matrices sorted by decreasing task count, so those with more than t tasks
// come first), i.e. task 0 (the POTRFs) of every matrix first, then task 1 of
// every matrix, and so on.  Each matrix's tasks keep their order, and the
// tasks of a column wait for the earlier columns' updates of their tiles
// through the per-block update counters (as in k_factor_all), so every task
// waits only for smaller tickets: the POTRF of column J0 + 1 starts as soon as
// column J0's updates of its tile are in, while the rest of column J0 goes on.
#define KB_COL_WG_PER_CU 2   // workgroups per compute unit of kb_column at tiles <= 128 (registers: 252 VGPRs)
#define KB_COL_MAX 16        // tile columns per kb_column launch, at most
struct BColArgs {
    const BInst* bi;
    const int* ints;                 // the queue tables
    int ncol;
    int tb[KB_COL_MAX + 1];          // first ticket of each column; tb[ncol]: all
    int off_at[KB_COL_MAX];          // ints + off_at[c]: off of column c, [T[c] + 1]
    int order_at[KB_COL_MAX];        // ints + order_at[c]: its matrices, by decreasing task count
    int T[KB_COL_MAX];               // most tasks of one matrix in column c
    int* ticket;
    int* err;                        // the batch's error word
    int64_t spin_limit;
};
// NPOOL = P3_POOL_128 when every tile of the batch is at most 128 wide: the
// smaller LDS footprint (49 KB against 147 KB) lets two workgroups share a
// compute unit, so the many small TRSM and update tasks of a column run twice
// as wide.
template <int NPOOL>
__global__ __launch_bounds__(P3_NT) void kb_column(BColArgs a, int64_t J0) {
    __shared__ ColSmemT<NPOOL> sm;
    __shared__ int sh;
    Sched sc;
    sc.ticket = a.ticket;
    sc.err = a.err;
    sc.spin_limit = a.spin_limit;
    sc.withhold = -1;
    for (;;) {
        const int g = sched_next(sc, a.tb[a.ncol], &sh);
        if (g < 0) return;
        int c = 0;
        while (c + 1 < a.ncol && g >= a.tb[c + 1]) ++c;
        const int gl = g - a.tb[c];
        const int* off = a.ints + a.off_at[c];
        int lo = 0, hi = a.T[c];
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (off[mid] <= gl) lo = mid; else hi = mid;
        }
        const int t = lo;
        const BInst& I = a.bi[a.ints[a.order_at[c] + gl - off[t]]];
        const int64_t J = J0 + c;
        const FactorWs f = factor_ws(I.L, I.ws);
        if (!col_task(sm, sh, I.Lm, I.L, J, f.Yd + J * (int64_t)I.L.b * 16, f.cf + J * col_stride(I.L), sc,
                      f.ldp + 2 * J, f.winfo, t, f.upd, g))
            return;
    }
}

__global__ __launch_bounds__(NT) void kb_zero_upper(BArgs a) {
    BATCH_DECODE(a, I, bid, nblk);
    zero_upper_body(I.Lm, I.L, bid);
}

// Corner POTRF (a_p <= 256) of the matrices listed in idx, one workgroup each.
__global__ __launch_bounds__(NT) void kb_corner(const BInst* bi, const int* idx) {
    extern __shared__ double smem[];
    const BInst& I = bi[idx[blockIdx.x]];
    const FactorWs f = factor_ws(I.L, I.ws);
    potrf_body(I.Lm + I.L.corner(), (int64_t)I.L.ap, I.L.ap, nullptr, 0, f.ldp + 2 * I.L.nt, f.winfo, I.L.nb, smem);
}

__global__ void kb_factor_final(const BInst* bi, const int* err) {
    if (threadIdx.x != 0) return;
    const BInst& I = bi[blockIdx.x];
    const FactorWs f = factor_ws(I.L, I.ws);
    factor_final_body(f.ldp, I.nparts, f.winfo, err, I.logdet, I.info);
}

// Selinv set-up of every matrix (one workgroup per matrix): info word and the
// Phase 2 ticket, error word, group offsets and counters.
__global__ __launch_bounds__(NT) void kb_selinv_setup(const BInst* bi) {
    const BInst& I = bi[blockIdx.x];
    const SelinvWs v = selinv_ws(I.L, I.ws);
    if (threadIdx.x == 0) *v.winfo = 0;
    p2_setup_body(make_p2(I.S, v, I.L, I.p2_tasks), v.ticket, v.err);
}

__global__ __launch_bounds__(NT) void kb_zero_unused(BArgs a) {
    BATCH_DECODE(a, I, bid, nblk);
    zero_unused_body(I.S, I.L, bid, nblk);
}

__global__ __launch_bounds__(NT) void kb_trtri(BArgs a) {
    __shared__ double smem[TRTRI_SMEM_DOUBLES];
    BATCH_DECODE(a, I, bid, nblk);
    const SelinvWs v = selinv_ws(I.L, I.ws);
    trtri_body(I.Lm, v.W, I.L, v.winfo, bid, smem);
}

__global__ __launch_bounds__(NT) void kb_trmm(BArgs a) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    BATCH_DECODE(a, I, bid, nblk);
    trmm_body(I.Lm, selinv_ws(I.L, I.ws).W, I.L, bid, smem);
}

__global__ __launch_bounds__(NT) void kb_lauum(BArgs a) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    BATCH_DECODE(a, I, bid, nblk);
    lauum_body(selinv_ws(I.L, I.ws).W, I.S, I.L, bid, smem);
}

// Phase 2 of every matrix in one persistent launch: each matrix runs on its
// own share of the workgroups, with its own tickets.
__global__ __launch_bounds__(NT) void kb_phase2(BArgs a) {
    __shared__ double smem[P2Cfg<P2_KC_BATCHED>::SMEM];
    __shared__ int sh[2];
    BATCH_DECODE(a, I, bid, nblk);
    const SelinvWs v = selinv_ws(I.L, I.ws);
    Sched sc;
    sc.ticket = v.ticket;
    sc.err = v.err;
    sc.spin_limit = a.spin_limit;
    sc.withhold = -1;
    p2_run<P2_KC_BATCHED>(make_p2(I.S, v, I.L, I.p2_tasks), sc, smem, sh);
}

__global__ void kb_selinv_final(const BInst* bi) {
    if (threadIdx.x != 0) return;
    const BInst& I = bi[blockIdx.x];
    const SelinvWs v = selinv_ws(I.L, I.ws);
    *(I.info + 1) = (*v.err != 0) ? *v.err : *v.winfo;
}

// ---------------------------------------------------------------------------
// Trace of a product over the tile pattern (gradient of log det)
// ---------------------------------------------------------------------------
// sum_ij S_ij B_ij over the real entries of two symmetric matrices stored on
// the same tile pattern: a diagonal band tile and the corner hold both
// triangles (weight 1 each), a band tile below the diagonal and an arrow tile
// the strictly lower part (weight 2: the upper part mirrors it); padding
// (rows or columns past nb in the band, past a in the arrow) is left out.
// Block g of TP_BLOCKS sums a contiguous range of the buffer in a fixed order
// into part[g]; k_trace_final adds the parts in order (Neumaier), so the
// result does not depend on timing.
#define TP_BLOCKS 1024
__global__ __launch_bounds__(NT) void k_trace_part(const double* __restrict__ S, const double* __restrict__ B, Lay L,
                                                   double* part) {
    __shared__ double red[NT];
    const int64_t per = (L.total + TP_BLOCKS - 1) / TP_BLOCKS;
    const int64_t lo = blockIdx.x * per, hi = std::min<int64_t>(L.total, lo + per);
    const int64_t b = L.b, b2 = b * b;
    double acc = 0.0;
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += NT) {
        double wgt = 0.0;
        if (idx < L.off_arrow) {
            const int64_t t = idx / b2, e = idx % b2;
            const int64_t J = t / (L.bt + 1), d = t % (L.bt + 1);
            const int64_t i = (J + d) * b + e % b, j = J * b + e / b;
            if (J + d < L.nt && i < L.nb && j < L.nb) wgt = d == 0 ? 1.0 : 2.0;
        } else if (idx < L.off_corner) {
            const int64_t e = idx - L.off_arrow;
            const int64_t J = e / ((int64_t)L.ap * b), f = e % ((int64_t)L.ap * b);
            if (f % L.ap < L.a && J * b + f / L.ap < L.nb) wgt = 2.0;
        } else {
            const int64_t e = idx - L.off_corner;
            if (e % L.ap < L.a && e / L.ap < L.a) wgt = 1.0;
        }
        if (wgt != 0.0) acc = fma(wgt * S[idx], B[idx], acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_trace_final(const double* part, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0, c = 0.0;
    for (int g = 0; g < TP_BLOCKS; ++g) neumaier(s, c, part[g]);
    *out = s + c;
}

// ---------------------------------------------------------------------------
// Selected entries read off the tile layout
// ---------------------------------------------------------------------------
// out[k] = Sigma(ij[2k], ij[2k+1]) (either order: Sigma is symmetric); NaN
// for a pair outside the tile pattern of L or outside the matrix.
__global__ __launch_bounds__(NT) void k_gather(const double* S, Lay L, const int64_t* ij, int64_t count, double* out) {
    const int64_t n = L.nb + L.a;
    for (int64_t k = blockIdx.x * (int64_t)NT + threadIdx.x; k < count; k += (int64_t)gridDim.x * NT) {
        int64_t i = ij[2 * k], j = ij[2 * k + 1];
        if (i < j) { const int64_t t = i; i = j; j = t; }
        double v = __builtin_nan("");
        if (j >= 0 && i < n) {
            if (j < L.nb) {
                const int64_t J = j / L.b, c = j - J * L.b;
                if (i < L.nb) {
                    const int64_t I = i / L.b;
                    if (I - J <= L.bt) v = S[L.band(J, (int)(I - J)) + (i - I * L.b) + c * L.b];
                } else {
                    v = S[L.arrow(J) + (i - L.nb) + c * L.ap];
                }
            } else {
                v = S[L.corner() + (i - L.nb) + (j - L.nb) * L.ap];
            }
        }
        out[k] = v;
    }
}

// ---------------------------------------------------------------------------
// Full inversion (every entry of A^{-1})
// ---------------------------------------------------------------------------
// The recurrence of Phase 2 taken over every tile row instead of the rows of
// S(J): in the padded index space (band rows 0 .. N b - 1, then the a_p arrow
// rows), with D the dense symmetric inverse (leading dimension np),
//   D[R, J] = -sum_{k in S(J)} D[R, k] Lhat_{k,J}   for all rows R below block J,
//   D[J, J] = X_J^T X_J - sum_{k in S(J)} Lhat_{k,J}^T D[k, J],
// for J = N-1 .. 0 after the corner D[A, A] = X_A^T X_A (Sec. III-D; the
// full-inversion case of Sec. III-B).  Only Lhat_{k,J} with k in S(J) is
// non-zero, so each block column is one product over the s band tiles and the
// arrow.  Every value goes to both triangles, so a later column reads D[i, k]
// for any i directly.

// Diagonal blocks X_J^T X_J (and the corner's) into D.
__global__ __launch_bounds__(NT) void k_inv_lauum(const double* W, double* D, int64_t ldd, Lay L) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    const int per = lauum_per(L);
    const int64_t nband = L.nt * (int64_t)per;
    const double* X;
    double* O;
    int m;
    int64_t ld;
    int t;
    if ((int64_t)blockIdx.x < nband) {
        const int64_t J = blockIdx.x / per;
        t = (int)(blockIdx.x % per);
        X = W + L.band(J, 0); m = L.b; ld = L.b;
        O = D + J * L.b + J * L.b * ldd;
    } else {
        t = (int)(blockIdx.x - nband);
        if (t >= lauum_corner(L)) return;
        X = W + L.corner(); m = L.ap; ld = L.ap;
        const int64_t o = L.nt * (int64_t)L.b;
        O = D + o + o * ldd;
    }
    int rb, cb;
    tri_decode(t, rb, cb);
    const int k0 = rb * 64;
    const int va = imin_(64, m - rb * 64), vb = imin_(64, m - cb * 64);
    GAcc g;
    gacc_zero(g);
    gemm_acc(g, opnd(X + k0 + (int64_t)rb * 64 * ld, ld, 1, va), opnd(X + k0 + (int64_t)cb * 64 * ld, ld, 0, vb),
             m - k0, smem);
    gemm_store_sym(g, smem, 1.0, 0.0, nullptr, 0, O + rb * 64 + (int64_t)cb * 64 * ldd,
                   O + cb * 64 + (int64_t)rb * 64 * ldd, ldd, rb == cb, va, vb);
}

// D[R, J] for the rows R = (J+1) b .. np-1; block (row block, column block)
// of 64 x 64, mirrored into D[J, R].
__global__ __launch_bounds__(NT) void k_inv_column(const double* W, double* D, int64_t ldd, Lay L, int64_t J) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    const int nb64 = L.b / 64;
    const int64_t r0 = (J + 1) * L.b;
    const int rbk = blockIdx.x / nb64, cb = blockIdx.x % nb64;
    const int64_t i0 = r0 + (int64_t)rbk * 64;
    const int mv = (int)std::min<int64_t>(64, ldd - i0);
    const int s = L.s(J);
    const int64_t ca = L.nt * (int64_t)L.b;   // first arrow column
    const int64_t c0 = J * L.b + cb * 64;
    GAcc g;
    gacc_zero(g);
    for (int d = 1; d <= s; ++d)
        gemm_acc(g, opnd(D + i0 + (J + d) * L.b * ldd, ldd, 0, mv), opnd(W + L.band(J, d) + (int64_t)cb * 64 * L.b, L.b, 0),
                 L.b, smem);
    if (L.ap > 0)
        gemm_acc(g, opnd(D + i0 + ca * ldd, ldd, 0, mv), opnd(W + L.arrow(J) + (int64_t)cb * 64 * L.ap, L.ap, 0),
                 L.ap, smem);
    gemm_store_sym(g, smem, -1.0, 0.0, nullptr, 0, D + i0 + c0 * ldd, D + c0 + i0 * ldd, ldd, 0, mv, 64);
}

// D[J, J] -= Lhat_{S,J}^T D[S, J], lower 64 x 64 blocks, mirrored.
__global__ __launch_bounds__(NT) void k_inv_diag(const double* W, double* D, int64_t ldd, Lay L, int64_t J) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    int rb, cb;
    tri_decode(blockIdx.x, rb, cb);
    const int s = L.s(J);
    const int64_t ca = L.nt * (int64_t)L.b;
    const int64_t j0 = J * L.b;
    GAcc g;
    gacc_zero(g);
    for (int d = 1; d <= s; ++d) {
        const double* Lh = W + L.band(J, d);
        gemm_acc(g, opnd(Lh + (int64_t)rb * 64 * L.b, L.b, 1), opnd(D + (J + d) * L.b + (j0 + cb * 64) * ldd, ldd, 0),
                 L.b, smem);
    }
    if (L.ap > 0) {
        const double* Lh = W + L.arrow(J);
        gemm_acc(g, opnd(Lh + (int64_t)rb * 64 * L.ap, L.ap, 1), opnd(D + ca + (j0 + cb * 64) * ldd, ldd, 0), L.ap,
                 smem);
    }
    double* O = D + j0 + j0 * ldd;
    gemm_store_sym(g, smem, -1.0, 1.0, O + rb * 64 + (int64_t)cb * 64 * ldd, ldd, O + rb * 64 + (int64_t)cb * 64 * ldd,
                   O + cb * 64 + (int64_t)rb * 64 * ldd, ldd, rb == cb, 64, 64);
}

// The real rows and columns of D into the n x n output (band index i -> i,
// arrow index nb + r -> N b + r).
__global__ __launch_bounds__(NT) void k_inv_compact(const double* D, int64_t ldd, Lay L, double* O) {
    const int64_t n = L.nb + L.a;
    const int64_t shift = L.nt * (int64_t)L.b - L.nb;
    for (int64_t idx = blockIdx.x * (int64_t)NT + threadIdx.x; idx < n * n; idx += (int64_t)gridDim.x * NT) {
        const int64_t i = idx % n, j = idx / n;
        const int64_t si = i < L.nb ? i : i + shift, sj = j < L.nb ? j : j + shift;
        O[idx] = D[si + sj * ldd];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Pure matrix-core throughput: every wavefront runs 8 independent chains of
// v_mfma_f64_16x16x4_f64 (2048 flops each), so the matrix pipe of its SIMD
// never waits on a result.  sink keeps the compiler from dropping the work.
#define PEAK_CHAINS 8
__global__ __launch_bounds__(NT) void k_mfma_peak(double* sink, int iters) {
    const int lane = threadIdx.x & 63;
    const double a = 1.0 + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
    dbl4 acc[PEAK_CHAINS];
#pragma unroll
    for (int c = 0; c < PEAK_CHAINS; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, (double)c};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < PEAK_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < PEAK_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    sink[blockIdx.x * (int64_t)NT + threadIdx.x] = s;
}

static inline hipStream_t S_(void* s) { return (hipStream_t)s; }

#define HIPCHK(x)                              \
    do {                                       \
        if ((x) != hipSuccess) return STILES_EHIP; \
    } while (0)
#define LAUNCHCHK()                                       \
    do {                                                  \
        if (hipGetLastError() != hipSuccess) return STILES_EHIP; \
    } while (0)


// Optional per-kernel event timing (see stiles_timing_enable in stiles.h).
struct EvRec {
    hipEvent_t a, b;
    int kind;
};
static std::mutex g_tmu;
static std::atomic<bool> g_timing{false};
static std::vector<EvRec> g_ev;

static hipEvent_t tm_begin(hipStream_t st) {
    if (!g_timing.load(std::memory_order_relaxed)) return nullptr;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    if (hipEventRecord(e, st) != hipSuccess) {
        (void)hipEventDestroy(e);
        return nullptr;
    }
    return e;
}

static void tm_end(hipEvent_t a, int kind, hipStream_t st) {
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> g(g_tmu);
    g_ev.push_back({a, b, kind});
}

static void tm_drop() {
    std::lock_guard<std::mutex> g(g_tmu);
    for (auto& e : g_ev) {
        (void)hipEventSynchronize(e.b);
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    g_ev.clear();
}

#define LAUNCH(kind, kern, grid, block, shm, st, ...)                           \
    do {                                                                       \
        hipEvent_t _tm = tm_begin(st);                                         \
        hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);           \
        if (hipGetLastError() != hipSuccess) return STILES_EHIP;               \
        tm_end(_tm, kind, st);                                                 \
    } while (0)

// Per-device facts used to size persistent launches (queried once).
struct DevInfo {
    int cus = 0;
    int64_t clock_khz = 0;
};
static std::mutex g_dmu;
static DevInfo g_dev[64];

static int dev_info(DevInfo* out) {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return STILES_EHIP;
    std::lock_guard<std::mutex> g(g_dmu);
    if (g_dev[d].cus == 0) {
        int cus = 0, khz = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess) return STILES_EHIP;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, d) != hipSuccess) return STILES_EHIP;
        g_dev[d].cus = cus > 0 ? cus : 1;
        g_dev[d].clock_khz = khz > 0 ? khz : 100000;
    }
    *out = g_dev[d];
    return 0;
}

// Wait limit of the device-side spin loops: STILES_SPIN_LIMIT_MS (default
// 4000 ms).  STILES_DEBUG_WITHHOLD=<ticket> makes that task skip its ready
// signal, to exercise the timeout path.
static int64_t spin_limit_ticks(const DevInfo& di) {
    double ms = 4000.0;
    if (const char* e = getenv("STILES_SPIN_LIMIT_MS")) {
        const double v = atof(e);
        if (v > 0) ms = v;
    }
    return (int64_t)(ms * (double)di.clock_khz);
}

// Tile columns per batched column launch: STILES_KB_COLS (1 .. KB_COL_MAX),
// default 8.  Measured on 64 matrices at tile 64: batched factor 64.4 / 55.6 /
// 52.1 / 49.9 / 49.1 ms at 1 / 2 / 4 / 8 / 16 columns per launch; served
// capacity (three concurrent lanes) 130 / 131 / 131 / 120 jobs/s at 1 / 4 / 8
// / 16, as a launch that holds every compute unit longer leaves the other
// lanes less room.
static int kb_cols_per_launch() {
    if (const char* e = getenv("STILES_KB_COLS")) {
        const int v = atoi(e);
        if (v >= 1 && v <= KB_COL_MAX) return v;
    }
    return 8;
}

static int debug_withhold() {
    if (const char* e = getenv("STILES_DEBUG_WITHHOLD")) return atoi(e);
    return -1;
}

static int grid_for(int64_t work) {
    int64_t g = (work + NT - 1) / NT;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// log det partial pairs: one per band tile column, one or two for the corner
static int factor_nparts(const Lay& L) {
    return (int)L.nt + (L.ap > 0 ? (L.ap <= 256 ? 1 : 2) : 0);
}

// The corner's Cholesky: one POTRF when a_p <= 256, else POTRF + TRTRI of
// its first 256 columns, TRSM and SYRK of the rest, POTRF of the remainder.
static int enqueue_corner(double* Lm, const Lay& L, const FactorWs& f, hipStream_t st) {
    if (L.ap == 0) return 0;
    double* Cc = Lm + L.corner();
    if (L.ap <= 256) {
        LAUNCH(STILES_TK_POTRF, k_potrf, dim3(1), dim3(NT), sizeof(double) * potrf_smem_doubles(L.ap), st, Cc,
               (int64_t)L.ap, L.ap, (double*)nullptr, (int64_t)0, f.ldp + 2 * L.nt, f.winfo, L.nb);
        return 0;
    }
    const int c2 = L.ap - 256;
    LAUNCH(STILES_TK_POTRF, k_potrf, dim3(1), dim3(NT), sizeof(double) * potrf_smem_doubles(256), st, Cc,
           (int64_t)L.ap, 256, f.Xc, (int64_t)256, f.ldp + 2 * L.nt, f.winfo, L.nb);
    LAUNCH(STILES_TK_OTHER, k_trsm_generic, dim3((c2 + 63) / 64), dim3(NT), 0, st, Cc + 256, (int64_t)L.ap, c2,
           (const double*)f.Xc, (int64_t)256, 256);
    const int nab2 = (c2 + 63) / 64;
    LAUNCH(STILES_TK_OTHER, k_syrk_generic, dim3(nab2 * (nab2 + 1) / 2), dim3(NT), 0, st,
           Cc + 256 + (int64_t)256 * L.ap, (int64_t)L.ap, (const double*)(Cc + 256), (int64_t)L.ap, c2, 256);
    LAUNCH(STILES_TK_POTRF, k_potrf, dim3(1), dim3(NT), sizeof(double) * potrf_smem_doubles(c2), st,
           Cc + 256 + (int64_t)256 * L.ap, (int64_t)L.ap, c2, (double*)nullptr, (int64_t)0, f.ldp + 2 * (L.nt + 1),
           f.winfo, L.nb + 256);
    LAUNCH(STILES_TK_OTHER, k_zero_block, dim3(64), dim3(NT), 0, st, Cc + (int64_t)256 * L.ap, (int64_t)L.ap, 256, c2);
    return 0;
}

static int64_t p2_total_tasks(const Lay& L) {
    int64_t t = 0;
    for (int64_t J = 0; J < L.nt; ++J) t += p2_group_tasks(L, J);
    return t;
}

// Batch plan: layouts, the table area at the start of the workspace (the
// matrices, then the launch segment tables) and each matrix's workspace.
static size_t align256(size_t x) { return (x + 255) / 256 * 256; }
struct BPlan {
    std::vector<stiles_layout> lay;
    std::vector<size_t> off;   // workspace offset of each matrix
    size_t table_f = 0;        // bytes of the factor's table area (at the start of the workspace)
    size_t table = 0;          // bytes of both table areas (the selected inverse's follows the factor's)
    size_t total = 0;
    int64_t maxN = 0;
};
// factor workspace (FactorWs): head (info, error words) + log det partials
// (N + 2 pairs) + the 256 x 256 inverse of the blocked corner + the 16 x 16
// diagonal-block inverses of every L_JJ + the per tile column counters.
static size_t fws_bytes(const stiles_layout& l) {
    const Lay L = to_dev(l);
    return WS_HEAD + sizeof(double) * (size_t)(2 * (l.nt + 2)) +
           sizeof(double) * (size_t)(256 * 256 + l.nt * (int64_t)l.tile * 16) +
           sizeof(int) * (size_t)(l.nt * (int64_t)col_stride(L) + upd_ints(L) + l.nt + 1);
}
// selinv workspace (SelinvWs): head (info, ticket, error words), the Phase 1
// tiles (inverted diagonal tiles, Lhat, corner inverse) in the tile layout,
// then the Phase 2 ready counters (P2_KINDS N).
static size_t sws_bytes(const stiles_layout& l) {
    return WS_HEAD + sizeof(double) * (size_t)l.total_doubles + sizeof(int) * (size_t)(P2_KINDS * l.nt);
}
static int batch_plan(const stiles_batch_item* items, int count, bool need_sigma, BPlan& pl) {
    pl.lay.resize(count);
    pl.off.resize(count);
    int64_t sumN = 0;
    for (int k = 0; k < count; ++k) {
        const stiles_batch_item& it = items[k];
        if (make_layout(it.n, it.bandwidth, it.arrow, it.tile, &pl.lay[k])) return -1;
        if (it.reserved != 0 || !it.A || !it.L || !it.logdet || !it.info) return -1;
        if (need_sigma && (!it.Sigma || it.Sigma == it.L)) return -1;
        if (need_sigma && p2_total_tasks(to_dev(pl.lay[k])) > 0x7fffffff) return -1;
        sumN += pl.lay[k].nt;
        pl.maxN = std::max(pl.maxN, pl.lay[k].nt);
    }
    // segment tables of at most six per-matrix launches; ints: the corner
    // list, the error word and a ticket per tile column, and the queue tables
    // of the tile-column launches (off: at most tmax + 1 per column; order:
    // sum of N)
    int64_t tmax = 0;
    for (int k = 0; k < count; ++k) {
        const Lay L = to_dev(pl.lay[k]);
        tmax = std::max<int64_t>(tmax, 1 + col_tr_blocks(L, 0) + col_up_blocks(L, 0));
    }
    const size_t nseg = 6 * ((size_t)count + 1);
    const size_t nint = (size_t)count + 1 + (size_t)pl.maxN + (size_t)pl.maxN * (size_t)(tmax + 1) + (size_t)sumN;
    pl.table_f = align256(sizeof(BInst) * (size_t)count) + align256(sizeof(BSeg) * nseg) + align256(sizeof(int) * nint);
    pl.table = pl.table_f + align256(sizeof(BInst) * (size_t)count) + align256(sizeof(BSeg) * nseg);
    size_t o = pl.table;
    for (int k = 0; k < count; ++k) {
        pl.off[k] = o;
        o += align256(std::max(fws_bytes(pl.lay[k]), sws_bytes(pl.lay[k])));
    }
    pl.total = o;
    return 0;
}

// Segment table builder: workgroup shares of one launch.
struct SegTab {
    std::vector<BSeg> v;
    size_t begin = 0;
    int grid = 0;
    void start(size_t b) { begin = b; grid = 0; }
    void add(std::vector<BSeg>& all, int inst, int blocks) {
        if (blocks <= 0) return;
        all.push_back({inst, grid});
        grid += blocks;
    }
    int finish(std::vector<BSeg>& all) {   // returns the segment count
        const int n = (int)(all.size() - begin);
        all.push_back({-1, grid});
        return n;
    }
};

extern "C" {

#ifdef STILES_TASK_TRACE
int stiles_debug_trace_read(unsigned long long* host, size_t n_tasks) {
    if (n_tasks > STILES_TRACE_MAX) n_tasks = STILES_TRACE_MAX;
    return hipMemcpyFromSymbol(host, HIP_SYMBOL(g_trace), STILES_TRACE_SLOTS * n_tasks * sizeof(unsigned long long), 0,
                               hipMemcpyDeviceToHost) == hipSuccess ? 0 : STILES_EHIP;
}
#endif

int stiles_version(void) { return 100; }

int stiles_timing_enable(int on) {
    tm_drop();
    g_timing.store(on != 0);
    return 0;
}

int stiles_timing_collect(double* ms, int64_t* launches) {
    if (!ms) return -1;
    if (!launches) return -2;
    for (int k = 0; k < STILES_TK_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    std::lock_guard<std::mutex> g(g_tmu);
    int rc = 0;
    for (auto& e : g_ev) {
        float t = 0.0f;
        if (hipEventSynchronize(e.b) != hipSuccess || hipEventElapsedTime(&t, e.a, e.b) != hipSuccess) rc = STILES_EHIP;
        if (e.kind >= 0 && e.kind < STILES_TK_COUNT) {
            ms[e.kind] += (double)t;
            launches[e.kind] += 1;
        }
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    g_ev.clear();
    return rc;
}


const char* stiles_strerror(int code) {
    if (code == 0) return "success";
    if (code > 0) return "matrix is not positive definite (info = failing column, 1-based)";
    switch (code) {
        case -1: return "invalid argument 1";
        case -2: return "invalid argument 2";
        case -3: return "invalid argument 3";
        case -4: return "invalid argument 4";
        case -5: return "invalid argument 5";
        case -6: return "invalid argument 6";
        case -7: return "invalid argument 7";
        case -8: return "invalid argument 8";
        case -9: return "invalid argument 9";
        case -10: return "invalid argument 10";
        case -11: return "invalid argument 11";
        case STILES_EHIP: return "HIP runtime error";
        case STILES_ETIMEOUT: return "device wait exceeded its spin limit";
        case STILES_EBADL: return "a diagonal entry of L is not positive";
        case STILES_ENOTBUILT: return "library not built or not loaded";
        default: return "invalid argument";
    }
}

int stiles_layout_init(int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile, stiles_layout* out) {
    if (!out) return -5;
    return make_layout(n, bandwidth, arrow, tile, out);
}

size_t stiles_factor_workspace_bytes(const stiles_layout* lay) { return lay ? fws_bytes(*lay) : 0; }

size_t stiles_selinv_workspace_bytes(const stiles_layout* lay) { return lay ? sws_bytes(*lay) : 0; }

int stiles_pack(const double* ab, const double* arrow_rows, const double* corner, double* tiles,
                int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile, void* stream) {
    stiles_layout lay;
    int rc = make_layout(n, bandwidth, arrow, tile, &lay);
    if (rc) return rc - 4;
    if (!ab) return -1;
    if (arrow > 0 && !arrow_rows) return -2;
    if (arrow > 0 && !corner) return -3;
    if (!tiles) return -4;
    Lay L = to_dev(lay);
    LAUNCH(STILES_TK_OTHER, k_pack, dim3((unsigned)(L.nt * (int64_t)(L.bt + 1) + L.nt + 1)), dim3(NT), 0, S_(stream),
           ab, arrow_rows, corner, tiles, L);
    return 0;
}

int stiles_factor(const double* A, double* Lm, int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile,
                  double* logdet, int32_t* info, void* workspace, size_t workspace_bytes, void* stream) {
    stiles_layout lay;
    int rc = make_layout(n, bandwidth, arrow, tile, &lay);
    if (rc) return rc - 2;
    if (!A) return -1;
    if (!Lm) return -2;
    if (!logdet) return -7;
    if (!info) return -8;
    if (!workspace || workspace_bytes < stiles_factor_workspace_bytes(&lay)) return -9;
    hipStream_t st = S_(stream);
    Lay L = to_dev(lay);
    const FactorWs f = factor_ws(L, (char*)workspace);
    const int cstride = col_stride(L);
    DevInfo di;
    if (dev_info(&di)) return STILES_EHIP;
    Sched sc;
    sc.ticket = nullptr;
    sc.err = f.err;
    sc.spin_limit = spin_limit_ticks(di);
    sc.withhold = debug_withhold();

    if (A != Lm) {
        hipEvent_t tm = tm_begin(st);
        HIPCHK(hipMemcpyAsync(Lm, A, sizeof(double) * (size_t)L.total, hipMemcpyDeviceToDevice, st));
        tm_end(tm, STILES_TK_OTHER, st);
    }
    LAUNCH(STILES_TK_OTHER, k_set_int, dim3(1), dim3(64), 0, st, f.winfo, 0x7fffffff);
    LAUNCH(STILES_TK_OTHER, k_set_int, dim3(1), dim3(64), 0, st, f.err, 0);
    LAUNCH(STILES_TK_OTHER, k_zero_ints, dim3(grid_for(L.nt * (int64_t)cstride + upd_ints(L))), dim3(NT), 0, st,
           f.cf, L.nt * (int64_t)cstride + upd_ints(L));
    LAUNCH(STILES_TK_OTHER, k_factor_offsets, dim3((unsigned)((L.nt + NT) / NT)), dim3(NT), 0, st, L, f.off, f.ticket);
    // One persistent launch: per tile column the POTRF of the diagonal tile,
    // the panel TRSM below it and the trailing updates, pipelined on the
    // 16-column panels, and the columns overlapped through the update
    // counters (k_factor_all).
    int64_t ntot = 0;
    for (int64_t J = 0; J < L.nt; ++J) ntot += 1 + col_tr_blocks(L, J) + col_up_blocks(L, J);
    if (ntot > 0x7fffffff) return -3;
    sc.ticket = f.ticket;
    LAUNCH(STILES_TK_FACTOR, k_factor_all, dim3((unsigned)std::min<int64_t>(ntot, di.cus)), dim3(P3_NT), 0, st, Lm, L,
           f.Yd, f.cf, f.upd, (const int*)f.off, sc, f.ldp, f.winfo);
    LAUNCH(STILES_TK_OTHER, k_zero_upper, dim3((unsigned)(8 * L.nt)), dim3(NT), 0, st, Lm, L);
    rc = enqueue_corner(Lm, L, f, st);
    if (rc) return rc;
    LAUNCH(STILES_TK_OTHER, k_factor_final, dim3(1), dim3(64), 0, st, (const double*)f.ldp, factor_nparts(L),
           (const int*)f.winfo, (const int*)f.err, logdet, (int*)info);
    return 0;
}

// Selected inverse on the tile columns J >= jf (and the corner): Phase 1 of
// the columns from jf - 1 on (the first Phase 2 group also holds the EA, E1A
// and EB tasks of column jf - 1), Phase 2 groups N-1 .. jf.  jf = 0 is the
// whole pattern.
static int selinv_impl(const double* Lm, double* S, const stiles_layout& lay, int64_t jf, int32_t* info,
                       void* workspace, hipStream_t st) {
    Lay L = to_dev(lay);
    const SelinvWs v = selinv_ws(L, (char*)workspace);
    const int nb64 = L.b / 64, nab = arrow_blocks(L.ap);
    int64_t ntasks = 0;
    for (int64_t J = jf; J < L.nt; ++J) ntasks += p2_group_tasks(L, J);
    if (ntasks > 0x7fffffff) return -3;
    const int64_t j1 = std::max<int64_t>(0, jf - 1);

    LAUNCH(STILES_TK_OTHER, k_set_int, dim3(1), dim3(64), 0, st, v.winfo, 0);
    if (L.bt > 0) {
        const int64_t tail = (int64_t)L.bt * (L.bt + 1) / 2 * L.b * L.b;
        LAUNCH(STILES_TK_OTHER, k_zero_unused, dim3(grid_for(tail)), dim3(NT), 0, st, S, L);
    }
    // Phase 1
    LAUNCH(STILES_TK_PHASE1, k_trtri_all, dim3((unsigned)(L.nt - j1 + (L.ap > 0))), dim3(NT), 0, st, Lm, v.W, L, v.winfo,
           j1);
    {
        const int64_t g = (L.nt - j1) * (int64_t)(L.bt * nb64 + nab) * nb64;
        if (g > 0) {
            LAUNCH(STILES_TK_PHASE1, k_trmm_all, dim3((unsigned)g), dim3(NT), 0, st, Lm, v.W, L, j1);
        }
    }
    {
        const int64_t g = lauum_blocks(L, j1);
        LAUNCH(STILES_TK_PHASE1, k_lauum_all, dim3((unsigned)g), dim3(NT), 0, st, (const double*)v.W, S, L, j1);
    }
    // Phase 2, bottom-right to top-left, one persistent launch
    DevInfo di;
    if (dev_info(&di)) return STILES_EHIP;
    const P2 p = make_p2(S, v, L, (int)ntasks);
    Sched sc;
    sc.ticket = v.ticket;
    sc.err = v.err;
    sc.spin_limit = spin_limit_ticks(di);
    sc.withhold = debug_withhold();
    LAUNCH(STILES_TK_OTHER, k_p2_setup, dim3(1), dim3(NT), 0, st, p, sc.ticket, sc.err);
    if (ntasks > 0) {
        const int grid = (int)std::min<int64_t>(ntasks, P2Cfg<P2_KC_SINGLE>::WG_PER_CU * (int64_t)di.cus);
        LAUNCH(STILES_TK_PHASE2, k_phase2, dim3(grid), dim3(NT), 0, st, p, sc);
    }
    LAUNCH(STILES_TK_OTHER, k_selinv_final, dim3(1), dim3(64), 0, st, (const int*)v.winfo, (const int*)v.err,
           (int*)info);
    return 0;
}

int stiles_selinv(const double* Lm, double* S, int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile,
                  int32_t* info, void* workspace, size_t workspace_bytes, void* stream) {
    stiles_layout lay;
    int rc = make_layout(n, bandwidth, arrow, tile, &lay);
    if (rc) return rc - 2;
    if (!Lm) return -1;
    if (!S || S == Lm) return -2;
    if (!info) return -7;
    if (!workspace || workspace_bytes < stiles_selinv_workspace_bytes(&lay)) return -8;
    return selinv_impl(Lm, S, lay, 0, info, workspace, S_(stream));
}

int stiles_selinv_range(const double* Lm, double* S, int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile,
                        int64_t first_column, int32_t* info, void* workspace, size_t workspace_bytes, void* stream) {
    stiles_layout lay;
    int rc = make_layout(n, bandwidth, arrow, tile, &lay);
    if (rc) return rc - 2;
    if (!Lm) return -1;
    if (!S || S == Lm) return -2;
    if (first_column < 0 || first_column > lay.nt) return -7;
    if (!info) return -8;
    if (!workspace || workspace_bytes < stiles_selinv_workspace_bytes(&lay)) return -9;
    return selinv_impl(Lm, S, lay, first_column, info, workspace, S_(stream));
}

int stiles_gather(const double* Sigma, int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile, const int64_t* ij,
                  int64_t count, double* out, void* stream) {
    stiles_layout lay;
    int rc = make_layout(n, bandwidth, arrow, tile, &lay);
    if (rc) return rc - 1;
    if (!Sigma) return -1;
    if (count < 0) return -7;
    if (count == 0) return 0;
    if (!ij) return -6;
    if (!out) return -8;
    LAUNCH(STILES_TK_OTHER, k_gather, dim3(grid_for(count)), dim3(NT), 0, S_(stream), Sigma, to_dev(lay), ij, count,
           out);
    return 0;
}

int stiles_selection_closure(int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile, const int64_t* ij,
                             int64_t count, int32_t* inside, int64_t* first_column) {
    stiles_layout lay;
    int rc = make_layout(n, bandwidth, arrow, tile, &lay);
    if (rc) return rc;
    if (count < 0) return -6;
    if (count > 0 && !ij) return -5;
    if (!inside) return -7;
    if (!first_column) return -8;
    const int64_t b = lay.tile, nb = lay.nb;
    int32_t in = 1;
    int64_t first = lay.nt;
    for (int64_t k = 0; k < count; ++k) {
        const int64_t i = ij[2 * k], j = ij[2 * k + 1];
        const int64_t hi = i > j ? i : j, lo = i > j ? j : i;
        if (lo < 0 || hi >= n) return -5;
        // a band entry lies in L's tile pattern when its tile row is within
        // B tiles of its tile column; arrow rows and the corner always do
        if (hi < nb && hi / b - lo / b > lay.bt) in = 0;
        const int64_t col = lo < nb ? lo / b : lay.nt;
        if (col < first) first = col;
    }
    *inside = in;
    *first_column = first;
    return 0;
}

int stiles_mfma_peak(double* sink, int64_t sink_doubles, int32_t iters, double* flops, void* stream) {
    if (!flops) return -4;
    if (iters < 1) return -3;
    DevInfo di;
    if (dev_info(&di)) return STILES_EHIP;
    const int64_t blocks = 2 * (int64_t)di.cus;
    if (!sink || sink_doubles < blocks * NT) return -1;
    *flops = (double)blocks * (NT / 64) * (double)iters * PEAK_CHAINS * 2048.0;
    hipLaunchKernelGGL(k_mfma_peak, dim3((unsigned)blocks), dim3(NT), 0, S_(stream), sink, (int)iters);
    LAUNCHCHK();
    return 0;
}

size_t stiles_trace_workspace_bytes(void) { return sizeof(double) * TP_BLOCKS; }

// padded order of the dense inverse: N b band rows and a_p arrow rows
static int64_t inv_order(const stiles_layout& l) { return l.nt * (int64_t)l.tile + l.arrow_ld; }

size_t stiles_inverse_workspace_bytes(const stiles_layout* lay) {
    if (!lay) return 0;
    const int64_t np = inv_order(*lay);
    return sws_bytes(*lay) + sizeof(double) * (size_t)(np * np);
}

int stiles_inverse(const double* Lm, double* Ainv, int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile,
                   int32_t* info, void* workspace, size_t workspace_bytes, void* stream) {
    stiles_layout lay;
    int rc = make_layout(n, bandwidth, arrow, tile, &lay);
    if (rc) return rc - 2;
    if (!Lm) return -1;
    if (!Ainv) return -2;
    if (!info) return -7;
    if (!workspace || workspace_bytes < stiles_inverse_workspace_bytes(&lay)) return -8;
    hipStream_t st = S_(stream);
    const Lay L = to_dev(lay);
    const SelinvWs v = selinv_ws(L, (char*)workspace);
    double* D = (double*)((char*)workspace + sws_bytes(lay));
    const int64_t np = inv_order(lay);
    const int nb64 = L.b / 64, nab = arrow_blocks(L.ap);

    LAUNCH(STILES_TK_OTHER, k_set_int, dim3(1), dim3(64), 0, st, v.winfo, 0);
    LAUNCH(STILES_TK_OTHER, k_set_int, dim3(1), dim3(64), 0, st, v.err, 0);
    LAUNCH(STILES_TK_OTHER, k_zero_ints, dim3(grid_for(np * np * 2)), dim3(NT), 0, st, (int*)D, np * np * 2);
    // Phase 1: X_J, Lhat (as for stiles_selinv)
    LAUNCH(STILES_TK_PHASE1, k_trtri_all, dim3((unsigned)(L.nt + (L.ap > 0))), dim3(NT), 0, st, Lm, v.W, L, v.winfo,
           (int64_t)0);
    {
        const int64_t g = L.nt * (int64_t)(L.bt * nb64 + nab) * nb64;
        if (g > 0) LAUNCH(STILES_TK_PHASE1, k_trmm_all, dim3((unsigned)g), dim3(NT), 0, st, Lm, v.W, L, (int64_t)0);
    }
    LAUNCH(STILES_TK_PHASE1, k_inv_lauum, dim3((unsigned)lauum_blocks(L, 0)), dim3(NT), 0,
           st, (const double*)v.W, D, np, L);
    for (int64_t J = L.nt - 1; J >= 0; --J) {
        const int64_t rows = np - (J + 1) * L.b;
        if (rows > 0) {
            const int64_t g = (rows + 63) / 64 * nb64;
            LAUNCH(STILES_TK_PHASE2, k_inv_column, dim3((unsigned)g), dim3(NT), 0, st, (const double*)v.W, D, np, L, J);
            LAUNCH(STILES_TK_PHASE2, k_inv_diag, dim3((unsigned)(nb64 * (nb64 + 1) / 2)), dim3(NT), 0, st,
                   (const double*)v.W, D, np, L, J);
        }
    }
    LAUNCH(STILES_TK_OTHER, k_inv_compact, dim3(grid_for(lay.n * lay.n)), dim3(NT), 0, st, (const double*)D, np, L,
           Ainv);
    LAUNCH(STILES_TK_OTHER, k_selinv_final, dim3(1), dim3(64), 0, st, (const int*)v.winfo, (const int*)v.err, (int*)info);
    return 0;
}

int stiles_trace_product(const double* Sigma, const double* B, int64_t n, int64_t bandwidth, int64_t arrow,
                         int32_t tile, double* out, void* workspace, size_t workspace_bytes, void* stream) {
    stiles_layout lay;
    int rc = make_layout(n, bandwidth, arrow, tile, &lay);
    if (rc) return rc - 2;
    if (!Sigma) return -1;
    if (!B) return -2;
    if (!out) return -7;
    if (!workspace || workspace_bytes < stiles_trace_workspace_bytes()) return -8;
    hipStream_t st = S_(stream);
    const Lay L = to_dev(lay);
    double* part = (double*)workspace;
    LAUNCH(STILES_TK_OTHER, k_trace_part, dim3(TP_BLOCKS), dim3(NT), 0, st, Sigma, B, L, part);
    LAUNCH(STILES_TK_OTHER, k_trace_final, dim3(1), dim3(64), 0, st, (const double*)part, out);
    return 0;
}

size_t stiles_batch_workspace_bytes(const stiles_batch_item* items, int32_t count) {
    if (!items || count < 1) return 0;
    BPlan pl;
    if (batch_plan(items, count, false, pl)) return 0;
    return pl.total;
}

// Host side of both batched calls: the matrix table (and the segment tables
// appended to `segs`) go to the table area of the workspace in one copy.
// Pinned host buffers for the table uploads, kept for the life of the
// process.  A buffer is handed out again only once the event recorded after
// its copy has completed, so calls on several streams at once (concurrent
// serving lanes) never overwrite a table that is still being copied.
struct PinnedBuf {
    char* p;
    size_t cap;
    hipEvent_t done;
};
static std::mutex g_pmu;
static std::vector<PinnedBuf> g_pin;
#define PIN_MAX_BUFS 16

// Host bytes -> device, through a pinned buffer, on stream st.
static int pinned_upload(void* dst, const void* src, size_t n, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_pmu);
    PinnedBuf* b = nullptr;
    for (auto& x : g_pin)
        if (x.cap >= n && hipEventQuery(x.done) == hipSuccess) {
            b = &x;
            break;
        }
    if (!b && g_pin.size() < PIN_MAX_BUFS) {
        PinnedBuf x;
        x.cap = std::max<size_t>(n, 1 << 16);
        HIPCHK(hipHostMalloc((void**)&x.p, x.cap, hipHostMallocDefault));
        if (hipEventCreateWithFlags(&x.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(x.p);
            return STILES_EHIP;
        }
        g_pin.push_back(x);
        b = &g_pin.back();
    }
    if (!b) {
        // every buffer busy: wait for the first one large enough, else grow it
        b = &g_pin[0];
        for (auto& x : g_pin)
            if (x.cap >= n) {
                b = &x;
                break;
            }
        HIPCHK(hipEventSynchronize(b->done));
        if (b->cap < n) {
            HIPCHK(hipHostFree(b->p));
            b->cap = n;
            HIPCHK(hipHostMalloc((void**)&b->p, b->cap, hipHostMallocDefault));
        }
    }
    memcpy(b->p, src, n);
    HIPCHK(hipMemcpyAsync(dst, b->p, n, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(b->done, st));
    return 0;
}

static int batch_upload(const std::vector<BInst>& bi, const std::vector<BSeg>& segs, const std::vector<int>& idx,
                        char* ws, hipStream_t st) {
    const size_t o1 = align256(sizeof(BInst) * bi.size()), o2 = o1 + align256(sizeof(BSeg) * 6 * (bi.size() + 1));
    std::vector<char> h(o2 + sizeof(int) * idx.size());
    memcpy(h.data(), bi.data(), sizeof(BInst) * bi.size());
    memcpy(h.data() + o1, segs.data(), sizeof(BSeg) * segs.size());
    if (!idx.empty()) memcpy(h.data() + o2, idx.data(), sizeof(int) * idx.size());
    return pinned_upload(ws, h.data(), h.size(), st);
}

// What a batched call does: upload its tables (host -> workspace, a copy
// from pageable memory staged before the call returns), enqueue its kernels
// (device work only, reading the tables; what a HIP graph can capture), or both.
#define BATCH_UPLOAD 1
#define BATCH_LAUNCH 2
static int factor_batched_impl(const stiles_batch_item* items, int32_t count, void* workspace,
                               size_t workspace_bytes, void* stream, int mode) {
    if (!items) return -1;
    if (count < 1) return -2;
    BPlan pl;
    if (batch_plan(items, count, false, pl)) return -1;
    if (!workspace) return -3;
    if (workspace_bytes < pl.total) return -4;
    hipStream_t st = S_(stream);
    DevInfo di;
    if (dev_info(&di)) return STILES_EHIP;
    char* ws = (char*)workspace;
    std::vector<BInst> bi(count);
    for (int k = 0; k < count; ++k) {
        BInst& I = bi[k];
        memset(&I, 0, sizeof(I));
        I.L = to_dev(pl.lay[k]);
        I.A = items[k].A;
        I.Lm = items[k].L;
        I.S = items[k].Sigma;
        I.logdet = items[k].logdet;
        I.info = items[k].info;
        I.ws = ws + pl.off[k];
        I.nparts = factor_nparts(I.L);
    }
    const size_t seg0 = align256(sizeof(BInst) * (size_t)count);
    const size_t int0 = seg0 + align256(sizeof(BSeg) * 6 * ((size_t)count + 1));
    std::vector<BSeg> segs;
    SegTab t;
    t.start(segs.size());
    for (int k = 0; k < count; ++k) t.add(segs, k, (int)(8 * bi[k].L.nt));
    const size_t zu_at = t.begin;
    const int zu_grid = t.grid, zu_n = t.finish(segs);
    // ints: [0, count) corner list, [count] error word, then one ticket per
    // tile column (zero as uploaded), then the queue tables
    std::vector<int> ints((size_t)count + 1 + (size_t)pl.maxN, 0);
    int ncorner = 0, corner_smem = 0;
    for (int k = 0; k < count; ++k)
        if (bi[k].L.ap > 0 && bi[k].L.ap <= 256) {
            ints[ncorner++] = k;
            corner_smem = std::max(corner_smem, (int)sizeof(double) * potrf_smem_doubles(bi[k].L.ap));
        }
    const size_t err_at = (size_t)count, tick_at = (size_t)count + 1;
    struct ColQ { size_t off_at, order_at; int T, ntot; };
    std::vector<ColQ> cq(pl.maxN);
    std::vector<std::pair<int, int>> nt_k;
    for (int64_t J = 0; J < pl.maxN; ++J) {
        nt_k.clear();
        for (int k = 0; k < count; ++k)
            if (bi[k].L.nt > J) nt_k.push_back({1 + col_tr_blocks(bi[k].L, J) + col_up_blocks(bi[k].L, J), k});
        std::stable_sort(nt_k.begin(), nt_k.end(), [](const std::pair<int, int>& x, const std::pair<int, int>& y) {
            return x.first > y.first;
        });
        ColQ& q = cq[J];
        q.T = nt_k.empty() ? 0 : nt_k.front().first;
        q.off_at = ints.size();
        int acc = 0;
        for (int tt = 0; tt <= q.T; ++tt) {
            ints.push_back(acc);
            for (const auto& e : nt_k) acc += e.first > tt;
        }
        q.ntot = acc;
        q.order_at = ints.size();
        for (const auto& e : nt_k) ints.push_back(e.second);
    }
    int rc = 0;
    if (mode & BATCH_UPLOAD) {
        rc = batch_upload(bi, segs, ints, ws, st);
        if (rc) return rc;
    }
    if (!(mode & BATCH_LAUNCH)) return 0;
    const BInst* dbi = (const BInst*)ws;
    const BSeg* dseg = (const BSeg*)(ws + seg0);
    int* dint = (int*)(ws + int0);
    const int64_t spin = spin_limit_ticks(di);

    // the error word and the tile-column tickets start at zero on every run
    LAUNCH(STILES_TK_OTHER, k_zero_ints, dim3(grid_for(1 + pl.maxN)), dim3(NT), 0, st, dint + err_at, 1 + pl.maxN);
    for (int k = 0; k < count; ++k) {
        if (bi[k].A == bi[k].Lm) continue;
        hipEvent_t tm = tm_begin(st);
        HIPCHK(hipMemcpyAsync(bi[k].Lm, bi[k].A, sizeof(double) * (size_t)bi[k].L.total, hipMemcpyDeviceToDevice, st));
        tm_end(tm, STILES_TK_OTHER, st);
    }
    LAUNCH(STILES_TK_OTHER, kb_factor_setup, dim3(count), dim3(NT), 0, st, dbi);
    int maxb = 0;
    for (int k = 0; k < count; ++k) maxb = std::max(maxb, bi[k].L.b);
    const int cols = kb_cols_per_launch();
    for (int64_t J0 = 0; J0 < pl.maxN; J0 += cols) {
        BColArgs a;
        memset(&a, 0, sizeof(a));
        a.bi = dbi;
        a.ints = dint;
        a.ncol = (int)std::min<int64_t>(cols, pl.maxN - J0);
        for (int c = 0; c < a.ncol; ++c) {
            const ColQ& q = cq[J0 + c];
            a.off_at[c] = (int)q.off_at;
            a.order_at[c] = (int)q.order_at;
            a.T[c] = q.T;
            a.tb[c + 1] = a.tb[c] + q.ntot;
        }
        a.ticket = dint + tick_at + J0;
        a.err = dint + err_at;
        a.spin_limit = spin;
        const int ntot = a.tb[a.ncol];
        if (maxb <= 128) {
            LAUNCH(STILES_TK_FACTOR, kb_column<P3_POOL_128>, dim3((unsigned)std::min(ntot, KB_COL_WG_PER_CU * di.cus)),
                   dim3(P3_NT), 0, st, a, J0);
        } else {
            LAUNCH(STILES_TK_FACTOR, kb_column<P3_POOL>, dim3((unsigned)std::min(ntot, di.cus)), dim3(P3_NT), 0, st, a,
                   J0);
        }
    }
    {
        const BArgs a{dbi, dseg + zu_at, zu_n, spin};
        LAUNCH(STILES_TK_OTHER, kb_zero_upper, dim3((unsigned)zu_grid), dim3(NT), 0, st, a);
    }
    if (ncorner > 0) {
        LAUNCH(STILES_TK_POTRF, kb_corner, dim3((unsigned)ncorner), dim3(NT), corner_smem, st, dbi, (const int*)dint);
    }
    for (int k = 0; k < count; ++k) {
        if (bi[k].L.ap <= 256) continue;
        rc = enqueue_corner(bi[k].Lm, bi[k].L, factor_ws(bi[k].L, bi[k].ws), st);
        if (rc) return rc;
    }
    LAUNCH(STILES_TK_OTHER, kb_factor_final, dim3(count), dim3(64), 0, st, dbi, (const int*)(dint + err_at));
    return 0;
}

static int selinv_batched_impl(const stiles_batch_item* items, int32_t count, void* workspace,
                               size_t workspace_bytes, void* stream, int mode) {
    if (!items) return -1;
    if (count < 1) return -2;
    BPlan pl;
    if (batch_plan(items, count, true, pl)) return -1;
    if (!workspace) return -3;
    if (workspace_bytes < pl.total) return -4;
    hipStream_t st = S_(stream);
    DevInfo di;
    if (dev_info(&di)) return STILES_EHIP;
    char* ws = (char*)workspace;
    char* tab = ws + pl.table_f;   // this call's table area
    std::vector<BInst> bi(count);
    int64_t sum_tasks = 0;
    for (int k = 0; k < count; ++k) {
        BInst& I = bi[k];
        memset(&I, 0, sizeof(I));
        I.L = to_dev(pl.lay[k]);
        I.A = items[k].A;
        I.Lm = items[k].L;
        I.S = items[k].Sigma;
        I.logdet = items[k].logdet;
        I.info = items[k].info;
        I.ws = ws + pl.off[k];
        I.p2_tasks = (int)p2_total_tasks(I.L);
        sum_tasks += I.p2_tasks;
    }
    const size_t seg0 = align256(sizeof(BInst) * (size_t)count);
    std::vector<BSeg> segs;
    SegTab t;
    struct Launch { size_t at; int n, grid; };
    auto close = [&](Launch& l) { l.at = t.begin; l.grid = t.grid; l.n = t.finish(segs); };
    Launch zu, tr, tm, la, p2;
    t.start(segs.size());
    for (int k = 0; k < count; ++k) {
        const Lay& L = bi[k].L;
        const int64_t tail = (int64_t)L.bt * (L.bt + 1) / 2 * L.b * L.b;
        if (L.bt > 0) t.add(segs, k, std::min(grid_for(tail), 256));
    }
    close(zu);
    t.start(segs.size());
    for (int k = 0; k < count; ++k) t.add(segs, k, (int)(bi[k].L.nt + (bi[k].L.ap > 0)));
    close(tr);
    t.start(segs.size());
    for (int k = 0; k < count; ++k) {
        const Lay& L = bi[k].L;
        const int nb64 = L.b / 64;
        t.add(segs, k, (int)(L.nt * (int64_t)(L.bt * nb64 + arrow_blocks(L.ap)) * nb64));
    }
    close(tm);
    t.start(segs.size());
    for (int k = 0; k < count; ++k) t.add(segs, k, (int)lauum_blocks(bi[k].L, 0));
    close(la);
    // Phase 2: the resident workgroups shared in proportion to the task
    // counts, at least one per matrix
    t.start(segs.size());
    {
        const int64_t total = std::min<int64_t>(sum_tasks, P2Cfg<P2_KC_BATCHED>::WG_PER_CU * (int64_t)di.cus);
        for (int k = 0; k < count; ++k) {
            const int64_t want = total * bi[k].p2_tasks / std::max<int64_t>(1, sum_tasks);
            t.add(segs, k, (int)std::max<int64_t>(1, std::min<int64_t>(bi[k].p2_tasks, want)));
        }
    }
    close(p2);
    if (mode & BATCH_UPLOAD) {
        const int rc = batch_upload(bi, segs, std::vector<int>(), tab, st);
        if (rc) return rc;
    }
    if (!(mode & BATCH_LAUNCH)) return 0;
    const BInst* dbi = (const BInst*)tab;
    const BSeg* dseg = (const BSeg*)(tab + seg0);
    const int64_t spin = spin_limit_ticks(di);
    auto args = [&](const Launch& l) { return BArgs{dbi, dseg + l.at, l.n, spin}; };

    LAUNCH(STILES_TK_OTHER, kb_selinv_setup, dim3(count), dim3(NT), 0, st, dbi);
    if (zu.grid > 0) LAUNCH(STILES_TK_OTHER, kb_zero_unused, dim3((unsigned)zu.grid), dim3(NT), 0, st, args(zu));
    LAUNCH(STILES_TK_PHASE1, kb_trtri, dim3((unsigned)tr.grid), dim3(NT), 0, st, args(tr));
    if (tm.grid > 0) LAUNCH(STILES_TK_PHASE1, kb_trmm, dim3((unsigned)tm.grid), dim3(NT), 0, st, args(tm));
    LAUNCH(STILES_TK_PHASE1, kb_lauum, dim3((unsigned)la.grid), dim3(NT), 0, st, args(la));
    LAUNCH(STILES_TK_PHASE2, kb_phase2, dim3((unsigned)p2.grid), dim3(NT), 0, st, args(p2));
    LAUNCH(STILES_TK_OTHER, kb_selinv_final, dim3(count), dim3(64), 0, st, dbi);
    return 0;
}

int stiles_factor_batched(const stiles_batch_item* items, int32_t count, void* workspace, size_t workspace_bytes,
                          void* stream) {
    return factor_batched_impl(items, count, workspace, workspace_bytes, stream, BATCH_UPLOAD | BATCH_LAUNCH);
}

int stiles_selinv_batched(const stiles_batch_item* items, int32_t count, void* workspace, size_t workspace_bytes,
                          void* stream) {
    return selinv_batched_impl(items, count, workspace, workspace_bytes, stream, BATCH_UPLOAD | BATCH_LAUNCH);
}

int stiles_batch_upload(const stiles_batch_item* items, int32_t count, void* workspace, size_t workspace_bytes,
                        void* stream) {
    const int rc = factor_batched_impl(items, count, workspace, workspace_bytes, stream, BATCH_UPLOAD);
    if (rc) return rc;
    return selinv_batched_impl(items, count, workspace, workspace_bytes, stream, BATCH_UPLOAD);
}

int stiles_factor_batched_enqueue(const stiles_batch_item* items, int32_t count, void* workspace,
                                  size_t workspace_bytes, void* stream) {
    return factor_batched_impl(items, count, workspace, workspace_bytes, stream, BATCH_LAUNCH);
}

int stiles_selinv_batched_enqueue(const stiles_batch_item* items, int32_t count, void* workspace,
                                  size_t workspace_bytes, void* stream) {
    return selinv_batched_impl(items, count, workspace, workspace_bytes, stream, BATCH_LAUNCH);
}

}  // extern "C"
