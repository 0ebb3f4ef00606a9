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

static Lay to_dev(const stiles_layout& s) {
    Lay l;
    l.nb = s.nb; l.w = s.w; l.nt = s.nt;
    l.off_band = s.off_band; l.off_arrow = s.off_arrow; l.off_corner = s.off_corner;
    l.total = s.total_doubles;
    l.b = s.tile; l.bt = s.bt; l.ap = s.arrow_ld; l.a = (int)s.arrow;
    return l;
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void k_set_int(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Pack the canonical band form into the tile layout (every double written).
__global__ __launch_bounds__(NT) void k_pack(const double* __restrict__ ab, const double* __restrict__ P,
                                            const double* __restrict__ C, double* __restrict__ T, Lay L) {
    const int64_t b = L.b, b2 = b * b;
    for (int64_t idx = blockIdx.x * (int64_t)NT + threadIdx.x; idx < L.total;
         idx += (int64_t)gridDim.x * NT) {
        double v = 0.0;
        if (idx < L.off_arrow) {
            const int64_t t = idx / b2, e = idx % b2;
            const int64_t J = t / (L.bt + 1), d = t % (L.bt + 1);
            const int64_t r = e % b, c = e / b;
            const int64_t i = (J + d) * b + r, j = J * b + c;
            if (J + d < L.nt) {
                if (i < L.nb && j < L.nb) {
                    const int64_t hi = i > j ? i : j, lo = i > j ? j : i;
                    if (hi - lo <= L.w) v = ab[(hi - lo) * L.nb + lo];
                } else if (i == j) {
                    v = 1.0;
                }
            }
        } else if (idx < L.off_corner) {
            const int64_t e = idx - L.off_arrow;
            const int64_t J = e / ((int64_t)L.ap * b), f = e % ((int64_t)L.ap * b);
            const int64_t r = f % L.ap, c = f / L.ap;
            const int64_t j = J * b + c;
            if (r < L.a && j < L.nb) v = P[r * L.nb + j];
        } else {
            const int64_t e = idx - L.off_corner;
            const int64_t r = e % L.ap, c = e / L.ap;
            if (r < L.a && c < L.a) v = C[r * L.a + c];
            else if (r == c) v = 1.0;
        }
        T[idx] = v;
    }
}

// Zero the band tiles (J+d, J) with J+d >= N (outside the matrix).
__global__ __launch_bounds__(NT) void k_zero_unused(double* T, Lay L) {
    const int64_t b2 = (int64_t)L.b * L.b;
    const int64_t ntail = (int64_t)L.bt * (L.bt + 1) / 2;  // tiles J+d >= N
    const int64_t tot = ntail * b2;
    for (int64_t idx = blockIdx.x * (int64_t)NT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * NT) {
        const int64_t t = idx / b2, e = idx % b2;
        // enumerate (J, d) with J = N-1-m, d = m+1..B, m = 0..B-1
        int64_t m = 0, cnt = t;
        while (cnt >= L.bt - m) { cnt -= L.bt - m; ++m; }
        const int64_t J = L.nt - 1 - m, d = m + 1 + cnt;
        T[L.band(J, (int)d) + e] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Factor kernels
// ---------------------------------------------------------------------------

// POTRF of one m x m diagonal block (m <= 256), optional TRTRI of the result
// into X, log det partial into ldp[0..1], first failing column into *info
// (atomicMin of the 1-based global column col_base + c + 1).
__global__ __launch_bounds__(NT) void k_potrf(double* M, int64_t ld, int m, double* X, int64_t ldx,
                                             double* ldp, int* info, int64_t col_base) {
    extern __shared__ double smem[];
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

// POTRF of one diagonal tile (m = b) plus the inverses of its 64 x 64
// diagonal blocks (for the panel TRSM): X64 + q*4096, 64 x 64 column-major.
__global__ __launch_bounds__(NT) void k_potrf_x64(double* M, int64_t ld, int m, double* X64, double* ldp, int* info,
                                                 int64_t col_base) {
    extern __shared__ double smem[];
    int fail;
    double s, c;
    potrf_tile(M, ld, m, smem, &fail, &s, &c);
    if (threadIdx.x == 0) {
        ldp[0] = s;
        ldp[1] = c;
        if (fail >= 0) atomicMin(info, (int)(col_base + fail + 1));
    }
    __syncthreads();
    inv64_blocks(M, ld, X64, m, smem);
}

// POTRF of one diagonal tile with the register-resident left-looking kernel
// (potrf3.hpp), plus the 64 x 64 diagonal-block inverses of L.
__global__ __launch_bounds__(NT) void k_potrf3(double* M, int64_t ld, int m, double* X64, double* ldp, int* info,
                                              int64_t col_base) {
    __shared__ P3Smem sm;
    int fail;
    double s, c;
    potrf3(M, ld, m, X64, sm, &fail, &s, &c);
    if (threadIdx.x == 0) {
        ldp[0] = s;
        ldp[1] = c;
        if (fail >= 0) atomicMin(info, (int)(col_base + fail + 1));
    }
}

// Strict upper triangles of the band diagonal tiles set to 0 (the layout's
// convention for L; k_potrf3 leaves them, as nothing in the factorization
// reads them).  Eight workgroups per tile, b/8 columns each.
__global__ __launch_bounds__(NT) void k_zero_upper(double* Lm, Lay L) {
    const int64_t J = blockIdx.x >> 3;
    const int cw = L.b / 8, c0 = (int)(blockIdx.x & 7) * cw;
    double* T = Lm + L.band(J, 0);
    for (int c = c0; c < c0 + cw; ++c)
        for (int i = threadIdx.x; i < c; i += NT) T[i + (int64_t)c * L.b] = 0.0;
}

// Panel TRSM, one 16-row block per workgroup: R = C L_JJ^{-T} in place, by
// forward substitution over the 64-column blocks q of the tile,
//   Z_q = C_q - sum_{q' < q} R_q' L_{q,q'}^T,   R_q = Z_q X64_q^T,
// with the transposed products formed on the matrix cores (Z^T = C^T - L R^T,
// R^T = X64 Z^T) so that every global access runs down a column.  Row block
// g0 + blockIdx.x of the rows below tile J: band tiles J+1..J+s (b/16 blocks
// each), then the arrow tile (a_p/16 blocks).  Wavefront w owns columns
// 64q + 16w .. 64q + 16w + 15 of each step.
#define TR_LD 16
#define TR_MAXA 48   // A operands of one step per lane: (b/64 - 1) * 16 for b = 256
__device__ inline void tr_bar_lds() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
__global__ __launch_bounds__(NT) void k_trsm16(double* Lm, Lay L, int64_t J, const double* X64, int g0) {
    __shared__ double sR[256 * TR_LD];   // R, [column][row]
    __shared__ double sZ[64 * TR_LD];    // Z of the current step, [column][row]
    const int g = g0 + blockIdx.x;
    const int nbr = L.b / 16, s = L.s(J);
    double* C;
    int ld;
    if (g < s * nbr) { C = Lm + L.band(J, 1 + g / nbr) + (g % nbr) * 16; ld = L.b; }
    else { C = Lm + L.arrow(J) + (g - s * nbr) * 16; ld = L.ap; }
    C = (double*)uniform_ptr(C);
    const double* Ljj = uniform_ptr(Lm + L.band(J, 0));
    const double* Xb = uniform_ptr(X64);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int b = L.b;
    const int nq = b / 64;
    const int KX = 16 * (w + 1);
    // operands of step 0 (C tile and X64 rows; no A operands yet)
    dbl4 cn;
    double xn[16];
#pragma unroll
    for (int r = 0; r < 4; ++r) cn[r] = ld_s(C, (uint32_t)(li + (16 * w + 4 * r + lk) * ld));
#pragma unroll
    for (int t = 0; t < 16; ++t) xn[t] = ld_s(Xb, (uint32_t)((16 * w + li) + (4 * t + lk) * 64));
    for (int q = 0; q < nq; ++q) {
        const int c0 = 64 * q + 16 * w;
        const int K = 64 * q;
        // Z^T tile (columns c0.., all 16 rows): element r = Z^T[4r + lk][li] = Z[li][c0 + 4r + lk]
        dbl4 a0 = cn, a1 = {0.0, 0.0, 0.0, 0.0};
        double xv[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) xv[t] = xn[t];
        double av[TR_MAXA];
#pragma unroll
        for (int t = 0; t < TR_MAXA; ++t)
            av[t] = -ld_s(Ljj, (uint32_t)((c0 + li) + imin_(4 * t + lk, b - 1) * b));
        // next step's C tile and X64 rows go out now
        if (q + 1 < nq) {
            const int c1 = c0 + 64;
#pragma unroll
            for (int r = 0; r < 4; ++r) cn[r] = ld_s(C, (uint32_t)(li + (c1 + 4 * r + lk) * ld));
#pragma unroll
            for (int t = 0; t < 16; ++t) xn[t] = ld_s(Xb, (uint32_t)((q + 1) * 4096 + (16 * w + li) + (4 * t + lk) * 64));
        }
#pragma unroll
        for (int t = 0; t < TR_MAXA; t += 2) {
            if (4 * t < K) {
                a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], sR[(4 * t + lk) * TR_LD + li], a0, 0, 0, 0);
                a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t + 1], sR[(4 * t + 4 + lk) * TR_LD + li], a1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sZ[(16 * w + 4 * r + lk) * TR_LD + li] = a0[r] + a1[r];
        tr_bar_lds();
        // R^T rows 16w.. of block q = X64_q(rows 16w..) Z^T; X64 is lower triangular
        dbl4 o0 = {0.0, 0.0, 0.0, 0.0}, o1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 16; t += 2) {
            if (4 * t < KX) {
                o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[t], sZ[(4 * t + lk) * TR_LD + li], o0, 0, 0, 0);
                o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[t + 1], sZ[(4 * t + 4 + lk) * TR_LD + li], o1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double v = o0[r] + o1[r];
            sR[(c0 + 4 * r + lk) * TR_LD + li] = v;
            st_s(C, (uint32_t)(li + (c0 + 4 * r + lk) * ld), v);
        }
        tr_bar_lds();   // sR and sZ reuse; the stores to C are read by no one here
    }
}

// Trailing update after tile column J on 32 x 32 blocks (reduction over the
// b columns of tile J spread over 4 wavefronts):
//   band (J+d, J+e), 1 <= e <= d <= s:  -= L_{J+d,J} L_{J+e,J}^T   (lower blocks when d == e)
//   arrow (A, J+e):                      -= L_{A,J} L_{J+e,J}^T
//   corner (lower blocks):               -= L_{A,J} L_{A,J}^T
__host__ __device__ inline int upd32_count(const Lay& L, int64_t J) {
    const int C32 = L.b / 32, s = L.s(J), na = (L.ap + 31) / 32;
    int cnt = 0;
    for (int d = 1; d <= s; ++d)
        for (int e = 1; e <= d; ++e) cnt += (d == e) ? C32 * (C32 + 1) / 2 : C32 * C32;
    if (L.ap > 0) cnt += s * na * C32 + na * (na + 1) / 2;
    return cnt;
}

__global__ __launch_bounds__(NT) void k_update32(double* Lm, Lay L, int64_t J, int t0) {
    __shared__ double smem[WS_SMEM_DOUBLES + 32 * WR_LD];
    double* red = smem + WS_SMEM_DOUBLES;
    const int C32 = L.b / 32, s = L.s(J), na = (L.ap + 31) / 32;
    int t = t0 + blockIdx.x;
    const double *Ap = nullptr, *Bp = nullptr;
    int64_t lda = L.b, ldb = L.b, ldo = L.b;
    int va = 32, vb = 32;
    double* O = nullptr;
    bool found = false;
    for (int d = 1; d <= s && !found; ++d) {
        for (int e = 1; e <= d && !found; ++e) {
            const int cnt = (d == e) ? C32 * (C32 + 1) / 2 : C32 * C32;
            if (t < cnt) {
                int rb, cb;
                if (d == e) tri_decode(t, rb, cb);
                else { rb = t % C32; cb = t / C32; }
                Ap = Lm + L.band(J, d) + rb * 32;
                Bp = Lm + L.band(J, e) + cb * 32;
                O = Lm + L.band(J + e, d - e) + rb * 32 + (int64_t)cb * 32 * L.b;
                found = true;
            } else {
                t -= cnt;
            }
        }
    }
    if (!found && L.ap > 0) {
        for (int e = 1; e <= s && !found; ++e) {
            const int cnt = na * C32;
            if (t < cnt) {
                const int rb = t % na, cb = t / na;
                Ap = Lm + L.arrow(J) + rb * 32; lda = L.ap; va = imin_(32, L.ap - rb * 32);
                Bp = Lm + L.band(J, e) + cb * 32;
                O = Lm + L.arrow(J + e) + rb * 32 + (int64_t)cb * 32 * L.ap; ldo = L.ap;
                found = true;
            } else {
                t -= cnt;
            }
        }
        if (!found) {
            int rb, cb;
            tri_decode(t, rb, cb);
            Ap = Lm + L.arrow(J) + rb * 32; lda = L.ap; va = imin_(32, L.ap - rb * 32);
            Bp = Lm + L.arrow(J) + cb * 32; ldb = L.ap; vb = imin_(32, L.ap - cb * 32);
            O = Lm + L.corner() + rb * 32 + (int64_t)cb * 32 * L.ap; ldo = L.ap;
        }
    }
    dbl4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    // the output block is read now, so its round trip overlaps the products
    double ov[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q, i = e & 31, j = e >> 5;
        ov[q] = (i < va && j < vb) ? O[i + (int64_t)j * ldo] : 0.0;
    }
    // B(k, j) = L_cols[j][k]: the transposed access of the column rows
    const Seg sg = mkseg(Ap, lda, 0, Bp, ldb, 1, L.b, va);
    wave_segs(acc, 1, L.b, smem, [&](int) { return sg; });
    wave_reduce(acc, smem, red);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q, i = e & 31, j = e >> 5;
        if (i < va && j < vb) O[i + (int64_t)j * ldo] = ov[q] - red[j * WR_LD + i];
    }
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
__global__ void k_factor_final(const double* ldp, int nparts, const int* info_ws, double* logdet,
                               int* info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0, c = 0.0;
    for (int i = 0; i < nparts; ++i) {
        neumaier(s, c, ldp[2 * i]);
        neumaier(s, c, ldp[2 * i + 1]);
    }
    const int f = *info_ws;
    *info = (f == 0x7fffffff) ? 0 : f;
    *logdet = (f == 0x7fffffff) ? (s + c) : __builtin_nan("");
}

// ---------------------------------------------------------------------------
// Selected-inversion kernels
// ---------------------------------------------------------------------------

// Phase 1, diagonal tiles: X_J = L_JJ^{-1} ("TRSM(L_ii^T, I)"), stored in the
// diagonal slots of the workspace; the corner inverse likewise.
__global__ __launch_bounds__(NT) void k_trtri_all(const double* Lm, double* W, Lay L, int* info) {
    __shared__ double smem[TRTRI_SMEM_DOUBLES];
    const int64_t J = blockIdx.x;
    int bad;
    if (J < L.nt) {
        trtri_tile(Lm + L.band(J, 0), L.b, W + L.band(J, 0), L.b, L.b, smem, &bad);
    } else {
        trtri_tile(Lm + L.corner(), L.ap, W + L.corner(), L.ap, L.ap, smem, &bad);
    }
    if (threadIdx.x == 0 && bad) atomicExch(info, STILES_EBADL);
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
__global__ __launch_bounds__(NT) void k_trmm_all(const double* Lm, double* W, Lay L) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    const int nb64 = L.b / 64;
    const int nab = arrow_blocks(L.ap);
    const int rows_max = L.bt * nb64 + nab;
    const int64_t J = blockIdx.x / (rows_max * nb64);
    const int r = (int)(blockIdx.x % (rows_max * nb64));
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

// Phase 2 initial value of each diagonal tile, "LAUUM": Sigma_JJ = X_J^T X_J
// (and the corner Sigma_AA = X_A^T X_A, which is final).  Lower 64 x 64
// blocks, mirrored so the tiles are full symmetric.
__global__ __launch_bounds__(NT) void k_lauum_all(const double* W, double* S, Lay L) {
    __shared__ double smem[GB_SMEM_DOUBLES];
    const int nb64 = L.b / 64;
    const int nab = arrow_blocks(L.ap);
    const int per = std::max(nb64 * (nb64 + 1) / 2, nab * (nab + 1) / 2);
    const int64_t J = blockIdx.x / per;
    const int t = blockIdx.x % per;
    const double* X;
    double* O;
    int m;
    int64_t ld;
    if (J < L.nt) {
        if (t >= nb64 * (nb64 + 1) / 2) return;
        X = W + L.band(J, 0); O = S + L.band(J, 0); m = L.b; ld = L.b;
    } else {
        if (t >= nab * (nab + 1) / 2) return;
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

#define ARW (-1)   // "the arrow" in place of a band tile offset

// ---------------------------------------------------------------------------
// Phase 2 as one persistent kernel
// ---------------------------------------------------------------------------
// Tile column J needs the off-diagonal tiles S(J) x S(J) of Sigma, where
// S(J) = band tiles J+1..J+s and the arrow.  Everything in S(J) x S(J) except
// what involves tile J+1 is final once column J+2 is done, so each output is
// split into an "early" part (k over the far tiles J+2..J+s and the arrow),
// which can start two columns ahead, and a "late" part (k = J+1).  Every task
// is a 32 x 32 block whose reduction is spread over the 4 wavefronts of a
// workgroup, so that the tasks on the dependency chain stay short:
//   E  : Sigma_{i,J}  = -sum_{k far} Sigma_{i,k} Lhat_{k,J}     i far
//   E1 : Sigma_{J+1,J} = -sum_{k far} Sigma_{J+1,k} Lhat_{k,J}
//   L  : Sigma_{i,J} -= Sigma_{i,J+1} Lhat_{J+1,J}               i far
//   L1 : Sigma_{J+1,J} -= Sigma_{J+1,J+1} Lhat_{J+1,J}
//   DA : Sigma_JJ = X_J^T X_J - sum_{i far} Lhat_{i,J}^T Sigma_{i,J}       (lower blocks)
//   DB : Sigma_JJ -= Lhat_{J+1,J}^T Sigma_{J+1,J}, then mirrored           (lower blocks)
// Dependencies (counters per tile column, "done(J)" = its last group):
//   E(J): done(J+2);  E1(J), L(J): off-diagonals of J+1 final (and E(J));
//   L1(J): Sigma_{J+1,J+1} final and E1(J);  DA(J): L(J);  DB(J): DA(J), L1(J).
// Ticket order: groups J = N-1 .. 0, group J = [E(J-1), E1(J), L(J), L1(J),
// DA(J), DB(J)] (group N-1 also starts with E(N-1)); every task depends only
// on tasks of earlier groups or earlier in its own group.
enum { P2_E = 0, P2_E1, P2_L, P2_L1, P2_DA, P2_DB, P2_KINDS };

struct P2 {
    double* S;
    const double* W;
    Lay L;
    int* group_off;  // [N+1]: first ticket of group J = N-1-q at group_off[q]
    int* cnt;        // [P2_KINDS * N] finished tasks per kind and tile column
    int ntasks;
};

struct P2Counts {
    int n[P2_KINDS];
};

// Task counts of tile column J.
__host__ __device__ inline P2Counts p2_counts(const Lay& L, int64_t J) {
    P2Counts c;
    const int s = L.s(J);
    const int C32 = L.b / 32;
    const int far = s > 1 ? s - 1 : 0;
    const int nf32 = far * C32 + (L.ap + 31) / 32;
    c.n[P2_E] = nf32 * C32;
    c.n[P2_E1] = s >= 1 ? C32 * C32 : 0;
    c.n[P2_L] = s >= 1 ? nf32 * C32 : 0;
    c.n[P2_L1] = s >= 1 ? C32 * C32 : 0;
    c.n[P2_DA] = C32 * (C32 + 1) / 2;
    c.n[P2_DB] = s >= 1 ? C32 * (C32 + 1) / 2 : 0;
    return c;
}

// Tasks in group J (see the ticket order above).
__host__ __device__ inline int p2_group_tasks(const Lay& L, int64_t J) {
    const P2Counts c = p2_counts(L, J);
    int t = c.n[P2_E1] + c.n[P2_L] + c.n[P2_L1] + c.n[P2_DA] + c.n[P2_DB];
    if (J >= 1) t += p2_counts(L, J - 1).n[P2_E];
    if (J == L.nt - 1) t += c.n[P2_E];
    return t;
}

__global__ void k_p2_setup(P2 p, int* ticket, int* err) {
    const Lay& L = p.L;
    for (int64_t i = threadIdx.x; i < P2_KINDS * L.nt; i += blockDim.x) p.cnt[i] = 0;
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int64_t q = 0; q < L.nt; ++q) {
            p.group_off[q] = acc;
            acc += p2_group_tasks(L, L.nt - 1 - q);
        }
        p.group_off[L.nt] = acc;
        *ticket = 0;
        *err = 0;
    }
}

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

// Is "done(J)" reached (all of column J final)?  Waits on the counters.
__device__ inline bool p2_wait_done(const P2& p, const Sched& sc, int64_t J, int* sh) {
    const P2Counts c = p2_counts(p.L, J);
    const int64_t N = p.L.nt;
    if (c.n[P2_DB] > 0) return sched_wait(sc, &p.cnt[P2_DB * N + J], c.n[P2_DB], sh);
    return sched_wait(sc, &p.cnt[P2_DA * N + J], c.n[P2_DA], sh);
}

// Are the off-diagonal tiles of column J final?
__device__ inline bool p2_wait_offdiag(const P2& p, const Sched& sc, int64_t J, int* sh) {
    const P2Counts c = p2_counts(p.L, J);
    const int64_t N = p.L.nt;
    if (c.n[P2_L1] > 0)
        return sched_wait(sc, &p.cnt[P2_L * N + J], c.n[P2_L], sh) &&
               sched_wait(sc, &p.cnt[P2_L1 * N + J], c.n[P2_L1], sh);
    return sched_wait(sc, &p.cnt[P2_E * N + J], c.n[P2_E], sh);
}

#define P2_SMEM_DOUBLES (WS_SMEM_DOUBLES + 32 * WR_LD)
#define P2_WG_PER_CU 2

// One Phase 2 task: a 32 x 32 output block, its reduction spread over the 4
// wavefronts.
__device__ __forceinline__ void p2_task_small(const P2& p, int kind, int64_t J, int u, bool mirror_da, double* smem,
                                           double* red, int t) {
    const Lay& L = p.L;
    const int C32 = L.b / 32;
    const int s = L.s(J);
    const int far = s > 1 ? s - 1 : 0;
    // output block and the reduction: L, L1, DB run over tile J+1 only (one
    // segment of b); DA over the far tiles and the arrow
    int d = 0, rbl = 0, rb = 0, cb = 0, nseg, ktot;
    const bool rowtask = kind <= P2_L1;            // E, E1, L, L1
    const bool kfar = kind == P2_E || kind == P2_E1;  // reduction over the far tiles
    if (rowtask) {
        if (kind == P2_E || kind == P2_L) p2_far_row(L, s, u / C32, 32, d, rbl);
        else { d = 1; rbl = u / C32; }
        cb = u % C32;
        nseg = kfar ? far + (L.ap > 0 ? 1 : 0) : 1;
        ktot = kfar ? far * L.b + L.ap : L.b;
    } else {
        tri_decode(u, rb, cb);
        nseg = (kind == P2_DA) ? far + (L.ap > 0 ? 1 : 0) : 1;
        ktot = (kind == P2_DA) ? far * L.b + L.ap : L.b;
    }
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
    // the partial already stored (L, L1, DB) is final once the task runs:
    // read it now so its round trip overlaps the products
    double ov[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q, i = e & 31, j = e >> 5;
        ov[q] = (kfar || i >= mv || (diag && i < j)) ? 0.0 : ld_coh(O + i + (int64_t)j * ldo);
    }
    dbl4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    wave_segs(acc, nseg, ktot, smem, [&](int q) {
        if (rowtask) {
            const int e = kfar ? ((q < far) ? q + 2 : ARW) : 1;
            const double* a; int64_t lda; int ta, av;
            p2_sigma_rows(L, p.S, J, d, rbl, 32, e, a, lda, ta, av);
            if (e != ARW)
                return mkseg(a, lda, ta, p.W + L.band(J, e) + (int64_t)cb * 32 * L.b, L.b, 0, L.b, av, 1, 0);
            return mkseg(a, lda, ta, p.W + L.arrow(J) + (int64_t)cb * 32 * L.ap, L.ap, 0, L.ap, av, 1, 0);
        }
        const int e = (kind == P2_DB) ? 1 : ((q < far) ? q + 2 : ARW);
        if (e != ARW)
            return mkseg(p.W + L.band(J, e) + (int64_t)rb * 32 * L.b, L.b, 1,
                         p.S + L.band(J, e) + (int64_t)cb * 32 * L.b, L.b, 0, L.b, 32, 0, 1);
        return mkseg(p.W + L.arrow(J) + (int64_t)rb * 32 * L.ap, L.ap, 1,
                     p.S + L.arrow(J) + (int64_t)cb * 32 * L.ap, L.ap, 0, L.ap, 32, 0, 1);
    });
    TRACE(t, 4, wall_clock64());
    wave_reduce(acc, smem, red);
    TRACE(t, 5, wall_clock64());
    // out = base - red, base = the partial already stored (L, L1, DB),
    // Sigma_JJ's initial value X^T X (DA), or 0 (E, E1)
    const bool mirror = (kind == P2_DB) || (kind == P2_DA && mirror_da);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + 256 * q, i = e & 31, j = e >> 5;
        if (i >= mv || (diag && i < j)) continue;
        red[j * WR_LD + i] = ov[q] - red[j * WR_LD + i];
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

__global__ __launch_bounds__(NT) void k_phase2(P2 p, Sched sc) {
    __shared__ double smem[P2_SMEM_DOUBLES];
    __shared__ int sh[2];
    double* red = smem + WS_SMEM_DOUBLES;
    const Lay& L = p.L;
    const int64_t N = L.nt;
    for (;;) {
        const int t = sched_next(sc, p.ntasks, &sh[0]);
        if (t < 0) break;
        TRACE(t, 0, wall_clock64());
        int lo = 0, hi = (int)N;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (p.group_off[mid] <= t) lo = mid; else hi = mid;
        }
        const int64_t G = N - 1 - lo;       // group
        int u = t - p.group_off[lo];
        // decode (kind, J, index) inside group G
        int kind = -1;
        int64_t J = G;
        {
            const P2Counts cg = p2_counts(L, G);
            if (G == N - 1) {
                if (u < cg.n[P2_E]) kind = P2_E;
                else u -= cg.n[P2_E];
            }
            if (kind < 0 && G >= 1) {
                const int ne = p2_counts(L, G - 1).n[P2_E];
                if (u < ne) { kind = P2_E; J = G - 1; }
                else u -= ne;
            }
            for (int k = P2_E1; kind < 0 && k < P2_KINDS; ++k) {
                if (u < cg.n[k]) kind = k;
                else u -= cg.n[k];
            }
        }
        const P2Counts c = p2_counts(L, J);
        int* my = &p.cnt[kind * N + J];

        // dependencies
        bool ok = true;
        switch (kind) {
            case P2_E: if (J + 2 < N) ok = p2_wait_done(p, sc, J + 2, &sh[1]); break;
            case P2_E1: ok = p2_wait_offdiag(p, sc, J + 1, &sh[1]); break;
            case P2_L:
                ok = p2_wait_offdiag(p, sc, J + 1, &sh[1]) && sched_wait(sc, &p.cnt[P2_E * N + J], c.n[P2_E], &sh[1]);
                break;
            case P2_L1:
                ok = p2_wait_done(p, sc, J + 1, &sh[1]) && sched_wait(sc, &p.cnt[P2_E1 * N + J], c.n[P2_E1], &sh[1]);
                break;
            case P2_DA:
                ok = (c.n[P2_L] > 0) ? sched_wait(sc, &p.cnt[P2_L * N + J], c.n[P2_L], &sh[1])
                                     : sched_wait(sc, &p.cnt[P2_E * N + J], c.n[P2_E], &sh[1]);
                break;
            default:
                ok = sched_wait(sc, &p.cnt[P2_DA * N + J], c.n[P2_DA], &sh[1]) &&
                     sched_wait(sc, &p.cnt[P2_L1 * N + J], c.n[P2_L1], &sh[1]);
        }
        if (!ok) break;
        TRACE(t, 1, wall_clock64());

        p2_task_small(p, kind, J, u, c.n[P2_DB] == 0, smem, red, t);
        sched_signal(sc, my, t);
        TRACE(t, 2, wall_clock64());
        TRACE(t, 3, (unsigned long long)kind | ((unsigned long long)J << 8) | ((unsigned long long)blockIdx.x << 40));
        TRACE(t, 7, (unsigned long long)__smid());
    }
}

__global__ void k_selinv_final(const int* info_ws, const int* err, int* info) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *info = (*err != 0) ? *err : *info_ws;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
#define WS_HEAD 256  // bytes reserved at the start of every workspace (info word)

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

// STILES_POTRF=1 selects the 16-panel right-looking diagonal-tile kernel
// instead of the default left-looking one (for comparisons).
static int g_potrf_kind = [] {
    const char* e = getenv("STILES_POTRF");
    return e ? atoi(e) : 0;
}();

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

// Two internal streams (default priority) and the events of the factor
// pipeline, one set per device, created on first use: the caller's stream
// forks into them and joins them back.  Running the chain on an internal
// stream rather than the caller's keeps the overlap when the caller uses the
// legacy default stream.  The mutex serialises the enqueue of concurrent
// factor calls on one device (their kernels may still overlap).
struct Side {
    hipStream_t a = nullptr, b = nullptr;
    hipEvent_t fork = nullptr, po = nullptr, tr = nullptr, up = nullptr, ja = nullptr, jb = nullptr;
    std::mutex mu;
};
static Side g_side[64];

static int side_get(Side** out) {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return STILES_EHIP;
    Side& sd = g_side[d];
    std::lock_guard<std::mutex> g(g_dmu);
    if (!sd.b) {
        hipStream_t a, b;
        if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess) return STILES_EHIP;
        // STILES_RESERVE_CUS=r keeps the off-chain stream off the first r
        // compute units, so the chain never waits for a free unit.
        int reserve = 0;
        if (const char* e = getenv("STILES_RESERVE_CUS")) reserve = atoi(e);
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess) return STILES_EHIP;
        if (reserve > 0 && reserve < cus) {
            std::vector<uint32_t> mask((cus + 31) / 32, 0u);
            for (int c = reserve; c < cus; ++c) mask[c / 32] |= 1u << (c % 32);
            if (hipExtStreamCreateWithCUMask(&b, (uint32_t)mask.size(), mask.data()) != hipSuccess) return STILES_EHIP;
        } else if (hipStreamCreateWithFlags(&b, hipStreamNonBlocking) != hipSuccess) {
            return STILES_EHIP;
        }
        hipEvent_t* ev[6] = {&sd.fork, &sd.po, &sd.tr, &sd.up, &sd.ja, &sd.jb};
        for (auto e : ev)
            if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return STILES_EHIP;
        sd.a = a;
        sd.b = b;
    }
    *out = &sd;
    return 0;
}

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

size_t stiles_factor_workspace_bytes(const stiles_layout* lay) {
    if (!lay) return 0;
    // head + log det partials (N + 2 blocks) + the 256 x 256 inverse of the
    // blocked corner + the 64 x 64 diagonal-block inverses of every L_JJ.
    return WS_HEAD + sizeof(double) * (size_t)(2 * (lay->nt + 2)) +
           sizeof(double) * (size_t)(256 * 256 + lay->nt * (int64_t)(lay->tile / 64) * 4096);
}

// selinv workspace: head (info, ticket, error words), the Phase 1 tiles
// (inverted diagonal tiles, Lhat, corner inverse) in the tile layout, then
// the Phase 2 step offsets and ready counters.
static size_t selinv_flags_ints(const stiles_layout* lay) { return (size_t)(7 * lay->nt + 1); }

size_t stiles_selinv_workspace_bytes(const stiles_layout* lay) {
    if (!lay) return 0;
    return WS_HEAD + sizeof(double) * (size_t)lay->total_doubles + sizeof(int) * selinv_flags_ints(lay);
}

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
    LAUNCH(STILES_TK_OTHER, k_pack, dim3(grid_for(L.total)), dim3(NT), 0, S_(stream), ab, arrow_rows, corner,
                       tiles, L);
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
    char* ws = (char*)workspace;
    int* winfo = (int*)ws;
    double* ldp = (double*)(ws + WS_HEAD);
    double* Xc = ldp + 2 * (L.nt + 2);
    double* X64 = Xc + 256 * 256;
    const int64_t x64_per = (int64_t)(L.b / 64) * 4096;
    Side* sd;
    if (side_get(&sd)) return STILES_EHIP;
    std::lock_guard<std::mutex> lk(sd->mu);
    hipStream_t sa = sd->a, sb = sd->b;

    if (A != Lm) {
        hipEvent_t tm = tm_begin(st);
        HIPCHK(hipMemcpyAsync(Lm, A, sizeof(double) * (size_t)L.total, hipMemcpyDeviceToDevice, st));
        tm_end(tm, STILES_TK_OTHER, st);
    }
    LAUNCH(STILES_TK_OTHER, k_set_int, dim3(1), dim3(64), 0, st, winfo, 0x7fffffff);
    // Two streams.  Stream a carries the dependency chain of the diagonal
    // tiles: POTRF(J) -> TRSM of tile (J+1, J) -> its SYRK into (J+1, J+1)
    // -> POTRF(J+1).  Stream b carries the rest of column J (TRSM of the
    // other rows, the other trailing updates), which overlaps the next steps
    // of the chain.
    HIPCHK(hipEventRecord(sd->fork, st));
    HIPCHK(hipStreamWaitEvent(sa, sd->fork, 0));
    HIPCHK(hipStreamWaitEvent(sb, sd->fork, 0));
    const size_t po_smem = sizeof(double) * potrf_smem_doubles(L.b);
    const int nbr = L.b / 16, C32 = L.b / 32;
    for (int64_t J = 0; J < L.nt; ++J) {
        const int s = L.s(J);
        double* Xj = X64 + J * x64_per;
        if (g_potrf_kind == 1)
            LAUNCH(STILES_TK_POTRF, k_potrf_x64, dim3(1), dim3(NT), po_smem, sa, Lm + L.band(J, 0), (int64_t)L.b, L.b,
                   Xj, ldp + 2 * J, winfo, J * (int64_t)L.b);
        else
            LAUNCH(STILES_TK_POTRF, k_potrf3, dim3(1), dim3(NT), 0, sa, Lm + L.band(J, 0), (int64_t)L.b, L.b, Xj,
                   ldp + 2 * J, winfo, J * (int64_t)L.b);
        HIPCHK(hipEventRecord(sd->po, sa));
        const int tr_crit = s >= 1 ? nbr : 0;
        const int tr_all = s * nbr + L.ap / 16;
        const int up_crit = s >= 1 ? C32 * (C32 + 1) / 2 : 0;
        const int up_all = upd32_count(L, J);
        if (tr_crit > 0) {
            if (J > 0) HIPCHK(hipStreamWaitEvent(sa, sd->up, 0));   // updates of column J-1 into tile (J+1, J)
            LAUNCH(STILES_TK_TRSM, k_trsm16, dim3(tr_crit), dim3(NT), 0, sa, Lm, L, J, (const double*)Xj, 0);
            HIPCHK(hipEventRecord(sd->tr, sa));
            LAUNCH(STILES_TK_UPDATE, k_update32, dim3(up_crit), dim3(NT), 0, sa, Lm, L, J, 0);
        }
        HIPCHK(hipStreamWaitEvent(sb, sd->po, 0));
        if (tr_all > tr_crit)
            LAUNCH(STILES_TK_TRSM, k_trsm16, dim3(tr_all - tr_crit), dim3(NT), 0, sb, Lm, L, J, (const double*)Xj,
                   tr_crit);
        if (tr_crit > 0) HIPCHK(hipStreamWaitEvent(sb, sd->tr, 0));
        if (up_all > up_crit)
            LAUNCH(STILES_TK_UPDATE, k_update32, dim3(up_all - up_crit), dim3(NT), 0, sb, Lm, L, J, up_crit);
        HIPCHK(hipEventRecord(sd->up, sb));
    }
    if (g_potrf_kind != 1)
        LAUNCH(STILES_TK_OTHER, k_zero_upper, dim3((unsigned)(8 * L.nt)), dim3(NT), 0, sb, Lm, L);
    HIPCHK(hipEventRecord(sd->ja, sa));
    HIPCHK(hipEventRecord(sd->jb, sb));
    HIPCHK(hipStreamWaitEvent(st, sd->ja, 0));
    HIPCHK(hipStreamWaitEvent(st, sd->jb, 0));
    int nparts = (int)L.nt;
    if (L.ap > 0) {
        double* Cc = Lm + L.corner();
        if (L.ap <= 256) {
            LAUNCH(STILES_TK_POTRF, k_potrf, dim3(1), dim3(NT), sizeof(double) * potrf_smem_doubles(L.ap), st, Cc,
                               (int64_t)L.ap, L.ap, (double*)nullptr, (int64_t)0, ldp + 2 * L.nt, winfo, L.nb);
            nparts += 1;
        } else {
            const int c2 = L.ap - 256;
            LAUNCH(STILES_TK_POTRF, k_potrf, dim3(1), dim3(NT), sizeof(double) * potrf_smem_doubles(256), st, Cc,
                               (int64_t)L.ap, 256, Xc, (int64_t)256, ldp + 2 * L.nt, winfo, L.nb);
            LAUNCH(STILES_TK_OTHER, k_trsm_generic, dim3((c2 + 63) / 64), dim3(NT), 0, st, Cc + 256, (int64_t)L.ap, c2,
                               (const double*)Xc, (int64_t)256, 256);
            const int nab2 = (c2 + 63) / 64;
            LAUNCH(STILES_TK_OTHER, k_syrk_generic, dim3(nab2 * (nab2 + 1) / 2), dim3(NT), 0, st,
                               Cc + 256 + (int64_t)256 * L.ap, (int64_t)L.ap, (const double*)(Cc + 256),
                               (int64_t)L.ap, c2, 256);
            LAUNCH(STILES_TK_POTRF, k_potrf, dim3(1), dim3(NT), sizeof(double) * potrf_smem_doubles(c2), st,
                               Cc + 256 + (int64_t)256 * L.ap, (int64_t)L.ap, c2, (double*)nullptr, (int64_t)0,
                               ldp + 2 * (L.nt + 1), winfo, L.nb + 256);
            LAUNCH(STILES_TK_OTHER, k_zero_block, dim3(64), dim3(NT), 0, st, Cc + (int64_t)256 * L.ap, (int64_t)L.ap,
                               256, c2);
            nparts += 2;
        }
    }
    LAUNCH(STILES_TK_OTHER, k_factor_final, dim3(1), dim3(64), 0, st, (const double*)ldp, nparts, (const int*)winfo,
                       logdet, (int*)info);
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
    hipStream_t st = S_(stream);
    Lay L = to_dev(lay);
    char* ws = (char*)workspace;
    int* winfo = (int*)ws;
    double* W = (double*)(ws + WS_HEAD);
    const int nb64 = L.b / 64, nab = arrow_blocks(L.ap);

    LAUNCH(STILES_TK_OTHER, k_set_int, dim3(1), dim3(64), 0, st, winfo, 0);
    if (L.bt > 0) {
        const int64_t tail = (int64_t)L.bt * (L.bt + 1) / 2 * L.b * L.b;
        LAUNCH(STILES_TK_OTHER, k_zero_unused, dim3(grid_for(tail)), dim3(NT), 0, st, S, L);
    }
    // Phase 1
    LAUNCH(STILES_TK_PHASE1, k_trtri_all, dim3((unsigned)(L.nt + (L.ap > 0))), dim3(NT), 0, st, Lm, W, L, winfo);
    {
        const int64_t g = L.nt * (int64_t)(L.bt * nb64 + nab) * nb64;
        if (g > 0) {
            LAUNCH(STILES_TK_PHASE1, k_trmm_all, dim3((unsigned)g), dim3(NT), 0, st, Lm, W, L);
        }
    }
    {
        const int per = std::max(nb64 * (nb64 + 1) / 2, nab * (nab + 1) / 2);
        const int64_t g = (L.nt + (L.ap > 0)) * (int64_t)per;
        LAUNCH(STILES_TK_PHASE1, k_lauum_all, dim3((unsigned)g), dim3(NT), 0, st, (const double*)W, S, L);
    }
    // Phase 2, bottom-right to top-left, one persistent launch
    {
        DevInfo di;
        if (dev_info(&di)) return STILES_EHIP;
        P2 p;
        p.S = S;
        p.W = W;
        p.L = L;
        int* fl = (int*)(W + L.total);
        p.group_off = fl;
        p.cnt = fl + L.nt + 1;
        int64_t ntasks = 0;
        for (int64_t J = 0; J < L.nt; ++J) ntasks += p2_group_tasks(L, J);
        if (ntasks > 0x7fffffff) return -3;
        p.ntasks = (int)ntasks;
        Sched sc;
        sc.ticket = winfo + 16;
        sc.err = winfo + 32;
        sc.spin_limit = spin_limit_ticks(di);
        sc.withhold = debug_withhold();
        LAUNCH(STILES_TK_OTHER, k_p2_setup, dim3(1), dim3(NT), 0, st, p, sc.ticket, sc.err);
        const int grid = (int)std::min<int64_t>(ntasks, P2_WG_PER_CU * (int64_t)di.cus);
        LAUNCH(STILES_TK_PHASE2, k_phase2, dim3(grid), dim3(NT), 0, st, p, sc);
    }
    LAUNCH(STILES_TK_OTHER, k_selinv_final, dim3(1), dim3(64), 0, st, (const int*)winfo, (const int*)(winfo + 32),
           (int*)info);
    return 0;
}

}  // extern "C"
