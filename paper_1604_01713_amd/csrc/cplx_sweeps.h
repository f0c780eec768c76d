// Complex (complex128) blocks on the FP64 matrix-core sweeps.
//
// A row-major n x P complex block with interleaved (re, im) entries is, as
// stored, a real n x 2P block whose column 2b is Re w_b and 2b+1 is Im w_b.
// Every contraction of a block step maps onto a real one of these views:
//   * Q^H W: with D = Q_r^T W_r (real, 2q x 2P),
//       Re (Q^H W)[c][b] = D[2c][2b] + D[2c+1][2b+1],
//       Im (Q^H W)[c][b] = D[2c][2b+1] - D[2c+1][2b]   (contraction);
//     W^H W the same way from the real Gram of W_r;
//   * W - Q S: W_r - Q_r S_r with the real 2q x 2P form of S,
//       S_r[2c][2b] = S_r[2c+1][2b+1] = Re s_cb,
//       S_r[2c][2b+1] = Im s_cb, S_r[2c+1][2b] = -Im s_cb   (expansion).
// The flop count is that of the complex products (four real multiply-adds
// per complex one).  Complex P = 8 runs on the 16-column real kernels with
// S expanded in memory; complex P = 16 (32 real columns) has the two sweeps
// below, which read S in its complex form and pick the real entry per lane.
#pragma once

#include "mfma_sweeps.h"

namespace bgcr {
namespace mx {

// ---------------------------------------------------------------------------
// Update sweep of 32-column FP64 blocks (complex P = 16): W'' = W - Q S with
// S complex (nq 16 x 16 blocks), stored (Wout non-null, in place allowed);
// with GRAM the partial 32 x 32 Gram W''^T W'' in part[wg][i 32 + j]; with
// NORM (Rinv, the complex 16 x 16 R^{-1}) V = W'' R^{-1} is stored instead,
// and there is no Gram.  As
// the 16-column update sweep with the D tile (W^T, 16 columns x 16 rows per
// wave) doubled: tile g holds columns 16 g .. 16 g + 15, and both share the
// Q operand loads (column-major, straight into registers).
// The A operand of the update is -S_r[c][w] for c = 4 kk + l / 16 (plus the
// block offset) and w = 16 g + l % 16: the lane reads the real or imaginary
// part of the complex entry (c / 2, w / 2) and applies its sign.
// ---------------------------------------------------------------------------
template <int NQ, bool GRAM, bool NORM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NQ <= 4 ? 1 : 2))) void k_update_wide(int64_t n, const double* Win, BlockPtrs Q, int nq,
                                                     const zd* __restrict__ S, double* Wout,
                                                     double* __restrict__ part, const zd* __restrict__ Rinv,
                                                     const Ctl* ctl, int step, int rev) {
    static_assert(!(GRAM && NORM), "a normalising sweep takes no Gram");
    using M = MX<double>;
    constexpr int P = 32, KK = 8, NQA = NQ > 0 ? NQ : 1, NQV = NQ * KK;
    if (ctl && ctl->active == 0 && !(ctl->meff == step && ctl->status == 0)) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double* Sc = (double*)smem;               // [NQA*16][16] complex S as (re, im), zero past nq*16 rows
    double* tr = Sc + NQA * 16 * 16 * 2;      // [4 waves][16][32]
    double* red = (double*)smem;              // reused by the Gram reduction at the end
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int bl = lane & 15, rq = lane >> 4;
    const double* Sd = (const double*)S;
    for (int e = t; e < NQA * 16 * 16 * 2; e += 256) Sc[e] = (e < nq * 16 * 16 * 2) ? Sd[e] : 0.0;
    // lane's entry of -S_r: real part where c and w have the same parity,
    // else the imaginary part, negated except for (c odd, w even)
    const int ol = (rq ^ bl) & 1;
    const double sg = ((rq & 1) && !(bl & 1)) ? 1.0 : -1.0;
    const int sbase = 2 * ((rq >> 1) * 16 + (bl >> 1)) + ol;
    const double* qb[NQA];
#pragma unroll
    for (int blk = 0; blk < NQA; ++blk) qb[blk] = (const double*)(blk < nq ? Q.p[blk] : Q.p[0]);
    // NORM: A operands (R^{-1}_r)^T[16 g + l % 16][4 kk + l / 16] = R^{-1}_r[4 kk + l / 16][16 g + l % 16],
    // the real form of the complex R^{-1} (real part where row and column have the same parity, else the
    // imaginary part, negated for (odd row, even column))
    double ra[2][KK];
    if constexpr (NORM) {
        const double* Rd = (const double*)Rinv;
        const double rsg = ((rq & 1) && !(bl & 1)) ? -1.0 : 1.0;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int kk = 0; kk < KK; ++kk)
                ra[g][kk] = rsg * Rd[2 * ((2 * kk + (rq >> 1)) * 16 + 8 * g + (bl >> 1)) + ol];
    }
    d4v gacc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) gacc[a][b] = d4v{0, 0, 0, 0};
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + MROWS - 1) / MROWS, lw, t0, t1);
    double* mytr = tr + wave * 16 * P;
    // W^T tiles in the D layout: tile g element v = W[row l % 16][16 g + drow(l, v)]
    auto load_w = [&](d4v (&w)[2], int64_t rbase) {
        const int64_t off = clamp_row(rbase + bl, n) * P;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int v = 0; v < 4; ++v) w[g][v] = Win[off + 16 * g + M::drow(lane, v)];
    };
    // column-major operands: [blk*KK + kk] holds Q_blk[rbase + l % 16][4 kk + l / 16]
    auto load_cr = [&](double (&qv)[NQA * KK], int64_t rbase) {
        const int64_t off = clamp_row(rbase + bl, n) * P + rq;
#pragma unroll
        for (int blk = 0; blk < NQ; ++blk)
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) qv[blk * KK + kk] = qb[blk][off + 4 * kk];
    };
    // up to 4 blocks the next tile's Q operands are loaded while the current
    // one is multiplied; beyond, the registers allow one set, and the second
    // resident workgroup of the CU overlaps its loads
    constexpr bool DB = NQ <= 4;
    double qn[NQA * KK];
    d4v wn[2] = {d4v{0, 0, 0, 0}, d4v{0, 0, 0, 0}};
    const int64_t cnt = t1 - t0, dstep = rev ? -MROWS : MROWS;
    if (cnt > 0) {
        const int64_t r0 = (rev ? t1 - 1 : t0) * MROWS + wave * 16;
        if constexpr (NQV > 0 && DB) load_cr(qn, r0);
        load_w(wn, r0);
    }
    __syncthreads();
#pragma unroll 1
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t tile = rev ? t1 - 1 - k : t0 + k;
        const int64_t rbase = tile * MROWS + wave * 16;
        d4v d[2] = {wn[0], wn[1]};
        // S is read from LDS in every tile (kept in registers across tiles it
        // would take 4 NQ KK of them)
        asm volatile("" ::: "memory");
        if constexpr (NQV > 0) {
            double qc[NQA * KK];
            if constexpr (DB) {
#pragma unroll
                for (int e = 0; e < NQV; ++e) qc[e] = qn[e];
                if (k + 1 < cnt) load_cr(qn, rbase + dstep);
            } else {
                load_cr(qc, rbase);
            }
#pragma unroll
            for (int blk = 0; blk < NQ; ++blk)
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const double* sp = Sc + sbase + 2 * (blk * 16 + 2 * kk) * 16;
#pragma unroll
                    for (int g = 0; g < 2; ++g) d[g] = M::mma(sg * sp[16 * g], qc[blk * KK + kk], d[g]);
                }
        }
        if (k + 1 < cnt) load_w(wn, rbase + dstep);
        const int64_t row = rbase + bl;
#pragma unroll
        for (int g = 0; g < 2; ++g) zero_tail<double>(d[g], rbase, n, lane);
        if constexpr (NORM) {
            // V^T = (R^{-1}_r)^T W''^T: B operand W''^T[4 kk + l/16][row l % 16] from the tile in LDS
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) mytr[bl * P + 16 * g + M::drow(lane, v)] = d[g][v];
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                d4v dv = d4v{0, 0, 0, 0};
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) dv = M::mma(ra[g][kk], mytr[bl * P + 4 * kk + rq], dv);
                if (row < n) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) Wout[row * P + 16 * g + M::drow(lane, v)] = dv[v];
                }
            }
        } else if (Wout && row < n) {
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) Wout[row * P + 16 * g + M::drow(lane, v)] = d[g][v];
        }
        if constexpr (GRAM) {
            // the tile, row-major 16 x 32, in the wave's LDS: both Gram operands
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) mytr[bl * P + 16 * g + M::drow(lane, v)] = d[g][v];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const double w0 = mytr[(4 * ks + rq) * P + bl];
                const double w1 = mytr[(4 * ks + rq) * P + 16 + bl];
                gacc[0][0] = M::mma(w0, w0, gacc[0][0]);
                gacc[0][1] = M::mma(w0, w1, gacc[0][1]);
                gacc[1][0] = M::mma(w1, w0, gacc[1][0]);
                gacc[1][1] = M::mma(w1, w1, gacc[1][1]);
            }
        }
    }
    if constexpr (GRAM) {
        // the four 16 x 16 tiles of the Gram, each summed over the waves in a
        // fixed order
#pragma unroll
        for (int g1 = 0; g1 < 2; ++g1)
#pragma unroll
            for (int g2 = 0; g2 < 2; ++g2) {
                __syncthreads();
#pragma unroll
                for (int v = 0; v < 4; ++v) red[(wave * 4 + v) * 64 + lane] = gacc[g1][g2][v];
                __syncthreads();
                const int v = t >> 6, l = t & 63;
                const double s = red[(0 * 4 + v) * 64 + l] + red[(1 * 4 + v) * 64 + l] +
                                 red[(2 * 4 + v) * 64 + l] + red[(3 * 4 + v) * 64 + l];
                const int i = M::drow(l, v), j = l & 15;
                part[(int64_t)lw * P * P + (16 * g1 + i) * P + 16 * g2 + j] = s;
            }
    }
}

// ---------------------------------------------------------------------------
// Dot sweep of one 32-column FP64 block W against [Q_0 .. Q_{nq-1}] (32-column
// blocks): partial D = Q^T W in part[wg][c 32 + w] (c < 32 nq).  The 2 nq
// chunks of 16 Q columns are split over the four waves (NCW each); every wave
// covers all rows of the workgroup's range, so its accumulators are complete
// partials (no cross-wave reduction) and each Q element is loaded once; the
// W rows are loaded by all four waves (the repeats hit the CU's cache).
// Operands A = W[row][w], B = Q[row][c] straight from global memory in their
// register layout (4 rows per instruction), double-buffered.
// ---------------------------------------------------------------------------
template <int NCW, int KS>
__global__ __launch_bounds__(256) void k_dot_wide(int64_t n, const double* __restrict__ W, BlockPtrs Q, int nq,
                                                  double* __restrict__ part, const Ctl* ctl, int rev) {
    using M = MX<double>;
    constexpr int P = 32, TROWS = 4 * KS;
    if (ctl && ctl->active == 0) return;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int q = nq * P, nc = 2 * nq, cl = lane & 15;
    const double* qp[NCW];
#pragma unroll
    for (int i = 0; i < NCW; ++i) {
        const int ch = wave * NCW + i;
        const int chv = ch < nc ? ch : 0;  // chunks past the last one repeat chunk 0 (never written)
        qp[i] = (const double*)Q.p[chv >> 1] + 16 * (chv & 1) + cl;
    }
    const double* wp[2] = {W + cl, W + 16 + cl};
    d4v acc[2][NCW];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int i = 0; i < NCW; ++i) acc[g][i] = d4v{0, 0, 0, 0};
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + TROWS - 1) / TROWS, lw, t0, t1);
    const int64_t cnt = t1 - t0, dstep = rev ? -TROWS : TROWS;
    auto load = [&](double (&qv)[KS][NCW], double (&wv)[KS][2], int64_t rbase) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int64_t off = clamp_row(rbase + 4 * ks + (lane >> 4), n) * P;
#pragma unroll
            for (int g = 0; g < 2; ++g) wv[ks][g] = wp[g][off];
#pragma unroll
            for (int i = 0; i < NCW; ++i) qv[ks][i] = qp[i][off];
        }
    };
    double qn[KS][NCW], wn[KS][2];
    if (cnt > 0) load(qn, wn, (rev ? t1 - 1 : t0) * TROWS);
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t rbase = (rev ? t1 - 1 - k : t0 + k) * TROWS;
        double qc[KS][NCW], wc[KS][2];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int g = 0; g < 2; ++g) wc[ks][g] = wn[ks][g];
#pragma unroll
            for (int i = 0; i < NCW; ++i) qc[ks][i] = qn[ks][i];
        }
        if (rbase + TROWS > n) {  // last, partial tile: rows past n contribute nothing
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int g = 0; g < 2; ++g) wc[ks][g] = rbase + 4 * ks + (lane >> 4) < n ? wc[ks][g] : 0.0;
        }
        if (k + 1 < cnt) load(qn, wn, rbase + dstep);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int i = 0; i < NCW; ++i) acc[g][i] = M::mma(wc[ks][g], qc[ks][i], acc[g][i]);
    }
    // accumulator [g][i] element v: W column 16 g + drow(l, v), Q column 16 (wave NCW + i) + l % 16
    const int64_t nout = (int64_t)q * P;
#pragma unroll
    for (int i = 0; i < NCW; ++i) {
        const int c = 16 * (wave * NCW + i) + cl;
        if (c < q) {
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) part[(int64_t)lw * nout + (int64_t)c * P + 16 * g + M::drow(lane, v)] = acc[g][i][v];
        }
    }
}

// ---------------------------------------------------------------------------
// Second pass of a block step for 32-column FP64 blocks (complex P = 16) in
// one sweep: W' = W - Q S (S complex, not stored) and the partial D = Q^T W'
// in part[wg][c 32 + w] (c < 32 nq).  The four waves of a workgroup share a
// 16-row tile and split the 2 nq chunks of 16 Q columns round-robin (wave w
// takes chunks w, w + 4, ...), so each Q element is loaded once:
//   * each wave forms the part of the update from its own chunks (column-major
//     Q operands straight from memory; wave 0 also adds W), and the four
//     partial W'^T tiles meet in LDS (one workgroup barrier per tile, slots
//     double-buffered);
//   * the wave's Q operands are turned into the row-major layout of the dot
//     product through a small wave-private LDS tile, and the wave takes the
//     dots of its chunks with the summed W' (A = W'[row][w], B = Q[row][c]).
// The next tile's operands are loaded while the current one waits at the
// barrier and takes its dots.
// ---------------------------------------------------------------------------
template <int NQ, bool GRAM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_proj_dot_wide(
    int64_t n, const double* __restrict__ Win, BlockPtrs Q, int nq, const zd* __restrict__ S,
    double* __restrict__ part, const Ctl* ctl, int rev) {
    using M = MX<double>;
    constexpr int P = 32, NC = 2 * NQ, NCW = (NC + 3) / 4, TS = 17;
    if (ctl && ctl->active == 0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double* Sc = (double*)smem;         // [NQ*16][16] complex S as (re, im)
    double* slot = Sc + NQ * 512;       // [2][4 waves][16 rows][32]: partial W' tiles
    double* tt = slot + 2 * 4 * 512;    // [4 waves][16][TS]: transpose tiles
    double* red = (double*)smem;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int bl = lane & 15, rq = lane >> 4;
    const int q = nq * P, nc = 2 * nq;
    const double* Sd = (const double*)S;
    for (int e = t; e < NQ * 512; e += 256) Sc[e] = (e < nq * 512) ? Sd[e] : 0.0;
    // lane's entry of -S_r (as in k_update_wide)
    const int ol = (rq ^ bl) & 1;
    const double sg = ((rq & 1) && !(bl & 1)) ? 1.0 : -1.0;
    const int sbase = 2 * ((rq >> 1) * 16 + (bl >> 1)) + ol;
    // the wave's chunks ch = wave + 4 i: column 16 (ch % 2) + l % 16 of block ch / 2
    const double* qp[NCW];
    int chw[NCW];
#pragma unroll
    for (int i = 0; i < NCW; ++i) {
        const int ch = wave + 4 * i;
        chw[i] = ch;
        const int chv = ch < nc ? ch : 0;
        qp[i] = (const double*)Q.p[chv >> 1] + 16 * (chv & 1);
    }
    d4v acc[2][NCW];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int i = 0; i < NCW; ++i) acc[g][i] = d4v{0, 0, 0, 0};
    // GRAM: wave w takes the tile (w / 2, w % 2) of the 32 x 32 Gram W'^T W'
    d4v gacc = d4v{0, 0, 0, 0};
    const int g1 = wave >> 1, g2 = wave & 1;
    const int lw = logical_wg();
    int64_t t0, t1;
    tile_span((n + 15) / 16, lw, t0, t1);
    const int64_t cnt = t1 - t0, dstep = rev ? -16 : 16;
    double* mytt = tt + wave * 16 * TS;
    // column-major operands of the update: [i][kk] = Q[rbase + l % 16][16 ch_i + 4 kk + l / 16]
    auto load_q = [&](double (&qv)[NCW][4], int64_t rbase) {
        const int64_t off = clamp_row(rbase + bl, n) * P + rq;
#pragma unroll
        for (int i = 0; i < NCW; ++i)
            if (chw[i] < nc) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) qv[i][kk] = qp[i][off + 4 * kk];
            }
    };
    // W^T tiles in the D layout (wave 0): tile g element v = W[row l % 16][16 g + drow(l, v)]
    auto load_w = [&](d4v (&w)[2], int64_t rbase) {
        const int64_t off = clamp_row(rbase + bl, n) * P;
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int v = 0; v < 4; ++v) w[g][v] = Win[off + 16 * g + M::drow(lane, v)];
    };
    double qc[NCW][4];
    d4v wn[2] = {d4v{0, 0, 0, 0}, d4v{0, 0, 0, 0}};
    if (cnt > 0) {
        const int64_t r0 = (rev ? t1 - 1 : t0) * 16;
        load_q(qc, r0);
        if (wave == 0) load_w(wn, r0);
    }
    __syncthreads();
#pragma unroll 1
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t rbase = (rev ? t1 - 1 - k : t0 + k) * 16;
        // S is read from LDS in every tile (not kept in registers)
        asm volatile("" ::: "memory");
        d4v d[2] = {wn[0], wn[1]};
#pragma unroll
        for (int i = 0; i < NCW; ++i)
            if (chw[i] < nc) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const double* sp = Sc + sbase + 2 * (8 * chw[i] + 2 * kk) * 16;
#pragma unroll
                    for (int g = 0; g < 2; ++g) d[g] = M::mma(sg * sp[16 * g], qc[i][kk], d[g]);
                }
            }
        // row-major dot operands of the wave's chunks: [i][ks] = Q[rbase + 4 ks + l / 16][16 ch_i + l % 16]
        double qr[NCW][4];
#pragma unroll
        for (int i = 0; i < NCW; ++i)
            if (chw[i] < nc) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) mytt[bl * TS + 4 * kk + rq] = qc[i][kk];
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) qr[i][ks] = mytt[(4 * ks + rq) * TS + bl];
            }
        if (k + 1 < cnt) {
            load_q(qc, rbase + dstep);
            if (wave == 0) load_w(wn, rbase + dstep);
        }
        double* sl = slot + (k & 1) * 4 * 512;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            zero_tail<double>(d[g], rbase, n, lane);
#pragma unroll
            for (int v = 0; v < 4; ++v) sl[wave * 512 + bl * P + 16 * g + M::drow(lane, v)] = d[g][v];
        }
        __syncthreads();
        // W'[rbase + 4 ks + l / 16][16 g + l % 16], the four partials added in order
        double wa[4][2];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int e = (4 * ks + rq) * P + 16 * g + bl;
                wa[ks][g] = ((sl[e] + sl[512 + e]) + sl[1024 + e]) + sl[1536 + e];
            }
#pragma unroll
        for (int i = 0; i < NCW; ++i)
            if (chw[i] < nc) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                    for (int g = 0; g < 2; ++g) acc[g][i] = M::mma(wa[ks][g], qr[i][ks], acc[g][i]);
            }
        if constexpr (GRAM) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                gacc = M::mma(g1 ? wa[ks][1] : wa[ks][0], g2 ? wa[ks][1] : wa[ks][0], gacc);
        }
    }
    // accumulator [g][i] element v: W column 16 g + drow(l, v), Q column 16 ch_i + l % 16
    (void)red;
    const int64_t nout = (int64_t)q * P, stride = nout + (GRAM ? P * P : 0);
#pragma unroll
    for (int i = 0; i < NCW; ++i) {
        const int c = 16 * chw[i] + bl;
        if (chw[i] < nc) {
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) part[(int64_t)lw * stride + (int64_t)c * P + 16 * g + M::drow(lane, v)] = acc[g][i][v];
        }
    }
    // Gram tile (g1, g2) element v: row 16 g1 + drow(l, v), column 16 g2 + l % 16, after the dots
    if constexpr (GRAM) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            part[(int64_t)lw * stride + nout + (16 * g1 + M::drow(lane, v)) * P + 16 * g2 + bl] = gacc[v];
    }
}

// S_r (2q x 2P, FP64, row-major) = real form of the complex q x P matrix S
__global__ void k_cx_expand(const zd* __restrict__ S, int q, int P, double* __restrict__ Sr, const Ctl* ctl) {
    if (ctl && ctl->active == 0) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= q * P) return;
    const int c = e / P, b = e % P, P2 = 2 * P;
    const zd s = S[e];
    Sr[(2 * c) * P2 + 2 * b] = s.x;
    Sr[(2 * c) * P2 + 2 * b + 1] = s.y;
    Sr[(2 * c + 1) * P2 + 2 * b] = -s.y;
    Sr[(2 * c + 1) * P2 + 2 * b + 1] = s.x;
}

// out (q x P complex) = (add ? add : 0) + sum over the nwg workgroup partials
// of the contraction of their real 2q x 2P matrices (part[wg stride + off +
// r 2P + s]), the complex entries summed over the workgroups in a fixed order
__global__ __launch_bounds__(256) void k_cx_reduce(const double* __restrict__ part, int nwg, int64_t stride, int64_t off,
                                                   int q, int P, const zd* __restrict__ add, zd* out, const Ctl* ctl) {
    if (ctl && ctl->active == 0) return;
    __shared__ zd red[256];
    const int t = threadIdx.x, o = blockIdx.x * 16 + (t % 16), g = t / 16;
    const int nout = q * P, P2 = 2 * P;
    // four partial sums per thread: four partials' loads in flight at once
    zd s4[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    if (o < nout) {
        const int c = o / P, b = o % P;
        const int64_t i00 = (int64_t)(2 * c) * P2 + 2 * b, i10 = i00 + P2;
        int w = g;
        for (; w + 16 * 3 < nwg; w += 16 * 4) {
            double a[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double* d = part + (int64_t)(w + 16 * u) * stride + off;
                a[u][0] = d[i00];
                a[u][1] = d[i10 + 1];
                a[u][2] = d[i00 + 1];
                a[u][3] = d[i10];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                s4[u].x += a[u][0] + a[u][1];
                s4[u].y += a[u][2] - a[u][3];
            }
        }
        for (; w < nwg; w += 16) {
            const double* d = part + (int64_t)w * stride + off;
            s4[0].x += d[i00] + d[i10 + 1];
            s4[0].y += d[i00 + 1] - d[i10];
        }
    }
    const zd s = {(s4[0].x + s4[1].x) + (s4[2].x + s4[3].x), (s4[0].y + s4[1].y) + (s4[2].y + s4[3].y)};
    red[t] = s;
    __syncthreads();
    if (t < 16 && o < nout) {
        zd r = add ? add[o] : zd{0.0, 0.0};
        for (int k = 0; k < 16; ++k) r += red[k * 16 + t];
        out[o] = r;
    }
}

// ---------------------------------------------------------------------------
template <bool GRAM, bool NORM = false>
hipError_t launch_update_wide_t(hipStream_t st, int64_t n, const double* Win, const BlockPtrs& Q, int nq,
                                const zd* S, double* Wout, double* part, int nwg, const Ctl* ctl, int step, bool rev,
                                const zd* Rinv = nullptr) {
#define L(NQ)                                                                                                      \
    case NQ: {                                                                                                     \
        const size_t lds = std::max((size_t)((NQ > 0 ? NQ : 1) * 512 + 4 * 16 * 32) * sizeof(double),             \
                                    (size_t)1024 * sizeof(double));                                                \
        hipLaunchKernelGGL((k_update_wide<NQ, GRAM, NORM>), dim3(nwg), dim3(256), lds, st, n, Win, Q, nq, S, Wout, \
                           part, Rinv, ctl, step, (int)rev);                                                       \
        break;                                                                                                     \
    }
    switch (nq) {
        L(1) L(2) L(3) L(4) L(5) L(6) L(7) L(8) L(9) L(10) L(11) L(12)
        default: return hipErrorNotSupported;
    }
#undef L
    return hipGetLastError();
}

template <bool GRAM>
hipError_t launch_proj_dot_wide(hipStream_t st, int64_t n, const double* Win, const BlockPtrs& Q, int nq,
                                const zd* S, double* part, int nwg, const Ctl* ctl, bool rev) {
#define L(NQ)                                                                                                      \
    case NQ: {                                                                                                     \
        const size_t lds = (size_t)(NQ * 512 + 2 * 4 * 512 + 4 * 16 * 17) * sizeof(double);                       \
        static std::once_flag fl;                                                                                  \
        std::call_once(fl, [] { allow_lds(k_proj_dot_wide<NQ, GRAM>); });                                          \
        hipLaunchKernelGGL((k_proj_dot_wide<NQ, GRAM>), dim3(nwg), dim3(256), lds, st, n, Win, Q, nq, S, part, ctl, \
                           (int)rev);                                                                              \
        break;                                                                                                     \
    }
    // (up to 10 blocks: beyond, the operands of the wave's chunks spill)
    switch (nq) {
        L(1) L(2) L(3) L(4) L(5) L(6) L(7) L(8) L(9) L(10)
        default: return hipErrorNotSupported;
    }
#undef L
    return hipGetLastError();
}

inline hipError_t launch_dot_wide(hipStream_t st, int64_t n, const double* W, const BlockPtrs& Q, int nq, double* part,
                                  int nwg, const Ctl* ctl, bool rev) {
    const int ncw = (2 * nq + 3) / 4;
#define L(NCW, KS)                                                                                                  \
    case NCW:                                                                                                       \
        hipLaunchKernelGGL((k_dot_wide<NCW, KS>), dim3(nwg), dim3(256), 0, st, n, W, Q, nq, part, ctl, (int)rev); \
        break;
    switch (ncw) {
        L(1, 4) L(2, 4) L(3, 4) L(4, 4) L(5, 2) L(6, 2)
        default: return hipErrorNotSupported;
    }
#undef L
    return hipGetLastError();
}

}  // namespace mx
}  // namespace bgcr
