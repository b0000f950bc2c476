// Size-tiered fused RSAI(tol) column kernel (gfx950, one wave per workgroup).
//
// A wave holds 64/G columns; each column is owned by an aligned group of G lanes.
// The dense LS block A(I_k, J_k) of eq. (2.3) lives in registers, row i of the block
// in lane (i mod G), register slot (i / G): a column's block is at most
// MMAX = G * RPL rows by QMAX columns. Index sets are LDS hash sets (global index ->
// local position); rows and columns are numbered in insertion order, new ones in
// ascending global order, so the block grows by appending rows at the bottom and
// columns at the right and the Householder factor can be updated in place
// (Algorithm 1, step 7): stored reflectors are applied to the new columns only,
// then new reflectors are formed.
//
// Every loop of Algorithm 1 runs in one pass of the wave's loop; groups that finish
// take the next column, so different groups of a wave may be at different loops.
// A column that outgrows the tier's caps is written to a spill record and resumed
// by the next larger tier.
#pragma once

#include "rsai_dev.h"

namespace rsai {

// Spill record: header of RHDR ints, then J (q), I (m), R (nR: dominant rows used so
// far), pending dominant rows (nRh). Header: [0] global column id, [1] matrix, [2] k,
// [3] l, [4] q, [5] m, [6] nR, [7] nRh, [8..9] flop count (double bits), [10] flags:
// bit 0 l is still to be advanced when the pending rows form J-hat, bit 1 the stored
// pattern is augmented but not yet solved, bit 2 dropping applies to that solve;
// [11] kept columns of the flop model of that solve, [12] the rows its kept factor
// was formed on.
constexpr int RHDR = 13;

template <int G_, int RPL_, int QMAX_, int STAGE_, int HSF_ = 2, int WPS_ = 2>
struct TierCfg {
    static constexpr int G = G_, RPL = RPL_, QMAX = QMAX_, STAGE = STAGE_;
    static constexpr int WPS = WPS_;  // waves per SIMD the register budget is cut for
    static constexpr int MMAX = G * RPL;
    static constexpr int GPW = 64 / G;
    static constexpr int LOGHSI = ilog2ceil(HSF_ * MMAX);  // row hash: HSF x MMAX slots
    static constexpr int HSI = 1 << LOGHSI;
    static constexpr int LOGHSJ = ilog2ceil(2 * QMAX);
    static constexpr int HSJ = 1 << LOGHSJ;
    static constexpr int NEWC = MMAX > QMAX ? MMAX : QMAX;
    static constexpr int RIN = HSI - MMAX - 1;  // candidates inserted per round (I)
    static constexpr int RJN = HSJ - QMAX - 1;  // (J)
    static constexpr int PREF = (QMAX > CMAX ? QMAX : CMAX) + 1;
    static constexpr int REC = RHDR + QMAX + MMAX + (MMAX + 1) + CMAX;  // spill record ints
    // small tiers keep a row of every column in registers for the residual of step 4
    // (all loads in flight together); larger tiers would spill those registers
    static constexpr bool FASTSEL = QMAX <= 12;
    static_assert(RPL <= 32 && QMAX <= 32, "bit masks");
    static_assert(RIN >= 1 && RJN >= 1, "hash sizes");
    static_assert(QMAX <= MMAX, "row j of the block must exist for every column j");
};

// Record layout (int32): [0] global column id, [1] matrix, [2] k, [3] l, [4] q, [5] m,
// [6] |R| (rows used as dominant rows, incl. k), [7] |R-hat| pending, [8..9] the
// column's flop count so far (double), [10] flags (bit 0: the loop counter is still
// to be advanced for the pending R-hat), then J[q], I[m], R[|R|], R-hat[|R-hat|].
// q = 0 and no pending R-hat means "start from scratch".
struct TierArgs {
    const MatDev *mats;
    int nmat;
    const int64_t *col_base;  // [nmat + 1]
    BuildParams P;
    ColOut out;
    int64_t arena_base;       // first arena slot of this tier
    int64_t qlen;             // tier 0: number of columns (all matrices)
    const int32_t *rec_in;    // tier >= 1: input records
    int rec_in_stride;
    const int32_t *rec_in_count;
    int64_t rec_in_cap;
    // Record queues of the later classes a spilled column may go to (index 0: the
    // next class). A column goes to the first class whose limits hold the estimated
    // |I_k| and |J_k| of its next augmentation, else to the last queue; nq = 0 means
    // no later class (a spill is then a cap error).
    static constexpr int MAXQ = 4;
    int nq;
    int32_t *q_rec[MAXQ];
    int q_stride[MAXQ];
    int32_t *q_count[MAXQ];
    int64_t q_cap[MAXQ];
    int q_mmax[MAXQ], q_qmax[MAXQ];
    int32_t *err;             // global error flags (bit 0: internal)
    int one_loop;             // 1: park every column after one loop (plain schedule)
    int sync_refill;          // 1: groups take new columns only when the whole wave is idle
};

// Per-group LDS. The staging tile doubles as scratch for the phase-local arrays:
// the new-entry lists and segment tables of the augmentation phases, and the
// residual accumulator and column order of the dominant-row phase.
template <class C>
struct GLds {
    double stage[C::STAGE * C::MMAX];
    double mt[C::QMAX];       // solution of the last LS solve, by column slot
    int64_t cb[C::QMAX];      // first entry of the column in each slot of J (CSC of A)
    int cl[C::QMAX];          // its length
    int Ilist[C::MMAX];
    int Jlist[C::QMAX];
    int hI[C::HSI];
    int hJ[C::HSJ];
    int Rh[CMAX];             // pending dominant rows
    int cnt;
    int fo_lo, fo_hi;         // factor record of a finished column (kept R)
    int pad;
    unsigned char hIv[C::HSI];  // local row of each key in hI

    // augmentation phases (K, C, D)
    __device__ int *newk() { return reinterpret_cast<int *>(stage); }
    __device__ int *news() { return newk() + C::NEWC; }
    __device__ int64_t *segb() { return reinterpret_cast<int64_t *>(stage + C::NEWC); }
    __device__ int *pref() { return reinterpret_cast<int *>(segb() + C::QMAX); }
    // dominant-row phase (J)
    __device__ double *racc() { return stage; }
    __device__ int *ord() { return reinterpret_cast<int *>(stage + C::MMAX); }

    static_assert(C::NEWC * 8 + C::QMAX * 8 + C::PREF * 4 <= C::STAGE * C::MMAX * 8, "scratch fits the tile");
    static_assert(C::MMAX * 8 + C::QMAX * 4 <= C::STAGE * C::MMAX * 8, "scratch fits the tile");
    static_assert(C::MMAX < 256, "local rows fit a byte");
};


// ----------------------------------------------------------------- tiers
// t0: up to 24 x 12 blocks (2D 5-point stencils), 8 columns per wave
// t1: up to 64 x 24 blocks (3D 7-point stencils), 4 columns per wave; one wave per
//     SIMD so that the fully unrolled QR keeps its 96 block entries per lane in
//     registers
// t2: up to 128 x 32 blocks, a whole wave per column (two rows per lane, the group
//     reductions crossing the 16-lane rows by permlane swaps): fully unrolled, its 64
//     block entries per lane stay in registers at one wave per SIMD
#ifndef RSAI_T0_STAGE
#define RSAI_T0_STAGE 6
#endif
#ifndef RSAI_T0_HSF
#define RSAI_T0_HSF 2
#endif
using Tier0 = TierCfg<8, 3, 12, RSAI_T0_STAGE, RSAI_T0_HSF>;
// tier 0 with hash tables of four times its row and column capacity (a tile choice of
// the autotuner: fewer probes per insertion, more slots cleared per column)
using Tier0H4 = TierCfg<8, 3, 12, RSAI_T0_STAGE, 4>;
using Tier1 = TierCfg<16, 4, 24, 8, 2, 1>;
using Tier2 = TierCfg<64, 2, 32, 8, 2, 1>;
void launch_tier2(const TierArgs &a, int waves, hipStream_t s);
void launch_tier0_h4(const TierArgs &a, int waves, hipStream_t s);

}  // namespace rsai
