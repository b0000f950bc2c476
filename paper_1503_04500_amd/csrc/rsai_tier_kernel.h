// Fused, size-tiered RSAI(tol) kernel: the whole loop of Algorithm 1 (Section 3)
// with the dropping of Section 4, for every column of one or more matrices.
// Included by the files that instantiate it for the size tiers (each tier's file is
// compiled with the unrolling it needs).
#pragma once
#include <climits>

#include "rsai_kernels.h"
#include "rsai_tier.h"

namespace rsai {


// The kernel's argument block in the kernarg segment, read through a pointer whose
// value the compiler cannot see: the fields the column loop needs only now and then
// (refill, spill, output) are loaded where they are used instead of being held in
// scalar registers across the loop.
__device__ __forceinline__ const __attribute__((address_space(4))) TierArgs *kargs() {
    const __attribute__((address_space(4))) TierArgs *p =
        (const __attribute__((address_space(4))) TierArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return p;
}

// MULTI = false: one matrix, whose pointers stay in scalar registers.
template <class C, bool MULTI>
__global__ __launch_bounds__(64, C::WPS) void tier_kernel(TierArgs args) {
    constexpr int G = C::G, RPL = C::RPL, QMAX = C::QMAX, MMAX = C::MMAX, GPW = C::GPW;
    constexpr int STAGE = C::STAGE;
    // columns per chunk of the QR update: the small first tier keeps one (a chunk may
    // reach past the wave's last column, which costs more there than the interleaving
    // saves)
    constexpr int QCB = QMAX <= 12 ? 1 : 4;
    constexpr int NRI = (C::RIN + G - 1) / G;   // per-lane candidates per I round
    constexpr int NRJ = (C::RJN + G - 1) / G;   // per-lane candidates per J round
    constexpr int NNEW = (C::NEWC + G - 1) / G;

    __shared__ GLds<C> lds[GPW];
    __shared__ FacChunk fch;
    const int lane = threadIdx.x;
    const int gl = lane % G;
    const int grp = lane / G;
    GLds<C> &S = lds[grp];
    const BuildParams P = args.P;
    if (*args.err & ERR_SKIP) return;  // the CSC contract failed: process nothing
    fac_chunk_init(fch);

    // ---- static, XCD-aware schedule: each of the 8 XCDs takes a contiguous range
    const bool first_tier = (args.rec_in == nullptr);
    const int64_t Q = first_tier ? args.qlen : min((int64_t)(*args.rec_in_count), args.rec_in_cap);
    const int nblk = gridDim.x;
    const int xcd = blockIdx.x % 8;
    const int widx = blockIdx.x / 8;
    const int nw = (nblk - xcd + 7) / 8;
    const int64_t chunk = (Q + 7) / 8;
    const int64_t qlo_range = (int64_t)xcd * chunk;
    const int64_t qhi_range = min(Q, qlo_range + chunk);
    const int64_t gstride = (int64_t)nw * GPW;
    int64_t u_next = qlo_range + (int64_t)widx * GPW + grp;

    // ---- per-group state (uniform inside a group)
    bool busy = false, fin = false;
    int64_t pos = 0;          // position in this launch's queue
    int64_t ucol = 0;         // global column id
    int mat = 0, k = 0;
    int q = 0, m = 0, l = 0, p = 0, qlo = 0;
    int qmod = 0;             // kept columns for the flop model of the next solve
    int mmod = 0;             // rows the kept factor of that model was formed on
    int kidx = -1;            // local row of k in I, or -1
    bool kR = false;          // k used as a dominant row while k is not in I
    int nRh = 0;
    bool solve = false, dropok = false, linc = true;
    bool park = false;        // plain schedule: write the state out after this loop
    int status = ST_OK;
    double rn = 0.0, fl = 0.0;
    MatDev A{};
    if constexpr (!MULTI) A = args.mats[0];
    // ---- per-lane block rows
    double b[RPL][QMAX];
    double y[RPL];
    double rd[RPL], bt[RPL];  // R(i,i) and beta_i of the reflectors of this lane's rows
    unsigned rflag = 0u;      // bit r: local row r*G+gl is in R (used dominant rows)

#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        y[r] = 0.0;
#pragma unroll
        for (int c = 0; c < QMAX; ++c) b[r][c] = 0.0;
    }

    while (true) {
        // ============================================================ A. refill
        bool start = false;
        // with sync_refill, groups of a wave start their columns together, so they
        // stay at the same loop and the wave's QR is only as wide as its work
        const bool may_refill = kargs()->sync_refill ? wave_all(!busy) : true;
        if (!busy && !fin && may_refill) {
            if (u_next < qhi_range) {
                pos = u_next;
                u_next += gstride;
                start = true;
            } else {
                fin = true;
            }
        }
        if (wave_all(fin)) break;

        const int32_t *rec = nullptr;
        if (start) {
            if (first_tier) {
                ucol = pos;
                if constexpr (MULTI) {
                    int lo = 0, hi = kargs()->nmat - 1;  // matrix with col_base[mat] <= ucol
                    while (lo < hi) {
                        int mid = (lo + hi + 1) / 2;
                        if (kargs()->col_base[mid] <= ucol) lo = mid; else hi = mid - 1;
                    }
                    mat = lo;
                    k = (int)(ucol - kargs()->col_base[mat]);
                } else {
                    mat = 0;
                    k = (int)ucol;
                }
            } else {
                rec = kargs()->rec_in + pos * (int64_t)kargs()->rec_in_stride;
                ucol = rec[0];
                mat = rec[1];
                k = rec[2];
            }
            if constexpr (MULTI) A = kargs()->mats[mat];
            busy = true;
            status = ST_OK;
            fl = 0.0;
            kR = false;
            kidx = -1;
            rn = 0.0;
            rflag = 0u;
            nRh = 0;
            for (int t = gl; t < C::HSI; t += G) S.hI[t] = HEMPTY;
            for (int t = gl; t < C::HSJ; t += G) S.hJ[t] = HEMPTY;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                y[r] = 0.0;
#pragma unroll
                for (int c = 0; c < QMAX; ++c) b[r][c] = 0.0;
            }
        }
        wave_sync();
        bool resumed = false;
        if (start) {
            int rq = 0, rm = 0, rl = 0, rnR = 0, rnRh = 0;
            if (rec) { rl = rec[3]; rq = rec[4]; rm = rec[5]; rnR = rec[6]; rnRh = rec[7]; }
            if (rq == 0 && rnRh == 0) {
                // fresh column: J = {k}, pending; I from column k (Algorithm 1, steps 1-2)
                q = 0; m = 0; l = 0; p = 1; qlo = 0; qmod = 0;
                solve = true; dropok = true; linc = true;
                if (gl == 0) {
                    S.Jlist[0] = k;
                    int sl;
                    hinsert<C::LOGHSJ>(S.hJ, k, sl);
                }
            } else {
                resumed = true;
                q = rq; m = rm; l = rl; p = 0; qlo = 0;
                linc = (rec[10] & 1) != 0;
                fl = __longlong_as_double(((long long)rec[9] << 32) | (long long)(unsigned)rec[8]);
                const int32_t *RJ = rec + RHDR;
                const int32_t *RI = RJ + rq;
                for (int t = gl; t < rq; t += G) {
                    int col = RJ[t];
                    S.Jlist[t] = col;
                    const int64_t b0 = A.colptr[col];
                    S.cb[t] = b0;
                    S.cl[t] = (int)(A.colptr[col + 1] - b0);
                    int sl;
                    hinsert<C::LOGHSJ>(S.hJ, col, sl);
                }
                for (int t = gl; t < rm; t += G) {
                    int row = RI[t];
                    S.Ilist[t] = row;
                    int sl;
                    hinsert<C::LOGHSI>(S.hI, row, sl);
                    if (sl >= 0) S.hIv[sl] = t;
                    if (row == k) kidx = t;
                }
                kidx = gmax_i<G>(kidx);
                nRh = rnRh;
                for (int t = gl; t < rnRh; t += G) S.Rh[t] = RI[rm + rnR + t];
            }
        }
        wave_sync();
        if (resumed) {
            // rows of R (the dominant rows used so far) -> flags of their local rows
            const int32_t *RR = rec + RHDR + q + m;
            const int nR = rec[6];
            for (int t = 0; t < nR; ++t) {
                int row = RR[t];
                int sl = hfind<C::LOGHSI>(S.hI, row);
                int li = sl >= 0 ? S.hIv[sl] : -1;
                if (li < 0 && row == k) kR = true;
                if (li >= 0 && (li % G) == gl) rflag |= 1u << (li / G);
            }
            // a resumed column is re-solved on its stored pattern
            solve = true;
            dropok = false;
        }

        // ====================================== K. J-hat from pending dominant rows
        // (Algorithm 1, step 5: columns of A(R-hat, :) not in J)
        bool spill = park;          // parked by the plain schedule: hand over as is
        int est_m = m, est_q = q;   // size estimate of a spilled column (routing)
        const bool parked = park;
        park = false;
        {
            const bool doK = busy && nRh > 0 && !spill;
            // start and prefix length of each pending row's pattern, held in registers
            // by every lane of the group (the loads are independent)
            int64_t sb[CMAX];
            int sp[CMAX + 1];
            sp[0] = 0;
#pragma unroll
            for (int t = 0; t < CMAX; ++t) {
                int64_t b0 = 0, e0 = 0;
                if (doK && t < nRh) {
                    const int rt = S.Rh[t];
                    b0 = A.rowptr[rt];
                    e0 = A.rowptr[rt + 1];
                }
                sb[t] = b0;
                sp[t + 1] = sp[t] + (int)(e0 - b0);
            }
            const int total = doK ? sp[CMAX] : 0;
            est_m = m;
            if (doK && gl == 0) S.cnt = 0;
            wave_sync();
            bool ovf = false;
            for (int base = 0; wave_any(doK && !ovf && base < total); base += C::RJN) {
                int cand[NRJ];
#pragma unroll
                for (int s = 0; s < NRJ; ++s) {
                    const int uu = base + s * G + gl;
                    cand[s] = -1;
                    if (doK && !ovf && uu < total && uu < base + C::RJN) {
                        int64_t b0 = sb[0];
                        int o0 = 0;
#pragma unroll
                        for (int t = 1; t < CMAX; ++t)
                            if (uu >= sp[t]) { b0 = sb[t]; o0 = sp[t]; }
                        cand[s] = A.colidx[b0 + (uu - o0)];
                    }
                }
#pragma unroll
                for (int s = 0; s < NRJ; ++s) {
                    if (cand[s] >= 0) {
                        int sl;
                        if (hinsert<C::LOGHSJ>(S.hJ, cand[s], sl)) {
                            int ps = atomicAdd(&S.cnt, 1);
                            if (ps < C::NEWC) S.newk()[ps] = cand[s];
                        }
                    }
                }
                wave_sync();
                if (doK && !ovf && q + S.cnt > QMAX) {
                    // |J-hat| extrapolated from the share of new columns seen so far
                    ovf = true;
                    est_q = q + (int)ceilf((float)S.cnt * (float)total / (float)min(base + C::RJN, total));
                }
                wave_sync();
            }
            const int nnew = (doK && !ovf) ? S.cnt : 0;
            if (doK) {
#pragma unroll
                for (int s = 0; s < NNEW; ++s) {
                    int idx = s * G + gl;
                    if (idx < nnew) {
                        int key = S.newk()[idx];
                        int rank = 0;
                        for (int t = 0; t < nnew; ++t) rank += (S.newk()[t] < key) ? 1 : 0;
                        S.Jlist[q + rank] = key;
                    }
                }
                if (linc) ++l;  // step 6
                if (ovf) {
                    spill = true;
                } else {
                    p = nnew;
                    if (linc && !resumed) {
                        // empty J-hat: the loop is consumed without a solve (step 6)
                        solve = (p > 0);
                        qlo = q;
                        qmod = q;
                        mmod = m;
                        dropok = true;
                    } else if (linc) {
                        // resumed by the plain schedule: the factor is rebuilt from the
                        // stored pattern; an empty J-hat still needs r for the next loop
                        solve = true;
                        qlo = 0;
                        dropok = (p > 0);
                        qmod = (p > 0) ? q : -1;
                        mmod = m;
                    } else {
                        // resumed column: its block is refactored from scratch here, but
                        // the method's work is the update from the stored pattern
                        solve = true;
                        qlo = 0;
                        dropok = (p > 0);
                        qmod = (p > 0) ? q : -1;
                        mmod = m;
                    }
                }
            }
            wave_sync();
        }

        // ================================ C. I-hat: rows of the new columns not in I
        {
            const bool doC = busy && !spill && p > 0;
            // pending columns in parallel: start -> LDS, length -> LDS, then every lane
            // forms the prefix in registers
            if (doC) {
                for (int t = gl; t < p; t += G) {
                    const int j = S.Jlist[q + t];
                    const int64_t b0 = A.colptr[j];
                    const int len = (int)(A.colptr[j + 1] - b0);
                    S.segb()[t] = b0;
                    S.pref()[t] = len;
                    S.cb[q + t] = b0;  // kept by slot for the gathers and the residual
                    S.cl[q + t] = len;
                }
                if (gl == 0) S.cnt = 0;
            }
            wave_sync();
            int cpx[QMAX + 1];
            cpx[0] = 0;
#pragma unroll
            for (int t = 0; t < QMAX; ++t) cpx[t + 1] = cpx[t] + ((doC && t < p) ? S.pref()[t] : 0);
            const int total = doC ? cpx[QMAX] : 0;
            bool ovf = false;
            for (int base = 0; wave_any(doC && !ovf && base < total); base += C::RIN) {
                int cand[NRI];
#pragma unroll
                for (int s = 0; s < NRI; ++s) {
                    const int uu = base + s * G + gl;
                    cand[s] = -1;
                    if (doC && !ovf && uu < total && uu < base + C::RIN) {
                        int seg = 0, o0 = 0;
#pragma unroll
                        for (int t = 1; t < QMAX; ++t)
                            if (uu >= cpx[t]) { seg = t; o0 = cpx[t]; }
                        cand[s] = A.rowidx[S.segb()[seg] + (uu - o0)];
                    }
                }
#pragma unroll
                for (int s = 0; s < NRI; ++s) {
                    if (cand[s] >= 0) {
                        int sl;
                        if (hinsert<C::LOGHSI>(S.hI, cand[s], sl)) {
                            int ps = atomicAdd(&S.cnt, 1);
                            if (ps < C::NEWC) { S.newk()[ps] = cand[s]; S.news()[ps] = sl; }
                        }
                    }
                }
                wave_sync();
                if (doC && !ovf && m + S.cnt > MMAX) {
                    // |I-hat| extrapolated from the share of new rows seen so far
                    ovf = true;
                    est_m = m + (int)ceilf((float)S.cnt * (float)total / (float)min(base + C::RIN, total));
                    est_q = q + p;
                }
                wave_sync();
            }
            if (doC && ovf) spill = true;
            // ============================ D. number the new rows (ascending order)
            const int nnew = (doC && !ovf) ? S.cnt : 0;
            int kpos = -1;
            if (doC && !ovf) {
#pragma unroll
                for (int s = 0; s < NNEW; ++s) {
                    int idx = s * G + gl;
                    if (idx < nnew) {
                        int key = S.newk()[idx];
                        int rank = 0;
                        for (int t = 0; t < nnew; ++t) rank += (S.newk()[t] < key) ? 1 : 0;
                        int li = m + rank;
                        S.Ilist[li] = key;
                        S.hIv[S.news()[idx]] = li;
                        if (key == k) kpos = li;
                    }
                }
            }
            kpos = gmax_i<G>(kpos);
            wave_sync();
            if (doC && !ovf) {
                if (kpos >= 0) {
                    kidx = kpos;
                    if (kR) {
                        if ((kpos % G) == gl) rflag |= 1u << (kpos / G);
                        kR = false;
                    }
                }
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    int i = r * G + gl;
                    if (i >= m && i < m + nnew) {
                        y[r] = (i == kidx) ? 1.0 : 0.0;
                    }
                }
                m += nnew;
            }
        }

        // ================================================ spill to the next tier
        if (wave_any(spill)) {
            int ps = 0;
            // destination class: the first whose limits hold the estimate
            int d = kargs()->nq - 1;
#pragma unroll
            for (int i = TierArgs::MAXQ - 2; i >= 0; --i)
                if (i < kargs()->nq - 1 && est_m <= kargs()->q_mmax[i] && est_q <= kargs()->q_qmax[i]) d = i;
            int32_t *qrec = kargs()->q_rec[0];
            int qstr = kargs()->q_stride[0];
            int64_t qcap = kargs()->q_cap[0];
            if (spill && gl == 0) ps = INT_MAX;
#pragma unroll
            for (int i = 0; i < TierArgs::MAXQ; ++i) {
                if (i > 0 && d == i) { qrec = kargs()->q_rec[i]; qstr = kargs()->q_stride[i]; qcap = kargs()->q_cap[i]; }
                // one counter address per pass, so that the lanes' increments combine
                const bool mine = spill && gl == 0 && d == i && i < kargs()->nq;
                if (wave_any(mine) && mine) ps = atomicAdd(kargs()->q_count[i], 1);
            }
            if (kargs()->nq <= 0) qrec = nullptr;
            ps = gbcast_i<G>(ps, gl == 0);
            // (the plain schedule parks every column that fits after each loop in queue
            // 0; a column that outgrew the class goes on to a later one)
            const bool ok = spill && qrec != nullptr && (int64_t)ps < qcap &&
                            (parked || !kargs()->one_loop || d > 0);
            int nR = __popc(rflag);
            nR = gsum_i<G>(nR) + (kR ? 1 : 0);
            if (spill && gl == 0) S.cnt = 0;
            wave_sync();
            if (ok) {
                int32_t *R = qrec + (int64_t)ps * qstr;
                if (gl == 0) {
                    R[0] = (int32_t)ucol; R[1] = mat; R[2] = k; R[3] = l;
                    R[4] = q; R[5] = m; R[6] = nR; R[7] = nRh;
                    const long long fb = __double_as_longlong(fl);
                    R[8] = (int32_t)(fb & 0xffffffffLL);
                    R[9] = (int32_t)(fb >> 32);
                    R[10] = parked ? 1 : 0;
                }
                for (int t = gl; t < q; t += G) R[RHDR + t] = S.Jlist[t];
                for (int t = gl; t < m; t += G) R[RHDR + q + t] = S.Ilist[t];
                int32_t *RR = R + RHDR + q + m;
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (rflag & (1u << r)) RR[atomicAdd(&S.cnt, 1)] = S.Ilist[r * G + gl];
                if (kR && gl == 0) RR[atomicAdd(&S.cnt, 1)] = k;
#pragma unroll
                for (int t = 0; t < CMAX; ++t)
                    if (t < nRh && gl == 0) RR[nR + t] = S.Rh[t];
            }
            if (spill && !ok) {
                // no larger tier can take the column
                status = ST_CAP;
                if (gl == 0 && qrec != nullptr && (int64_t)ps >= qcap) atomicOr(kargs()->err, 32);  // queue full
            }
            if (spill && ok) busy = false;
            wave_sync();
        }
        if (busy && !spill) nRh = 0;  // pending rows consumed

        // ============================================ LS solve(s): gather + QR
        // pass 0: the augmented pattern (or the stored pattern of a resumed column);
        // pass 1: the pattern kept after dropping (Section 4).
        bool singular = false;
        bool redo = false;
#pragma unroll 1
        for (int pass = 0; pass < 2; ++pass) {
            const bool act = busy && status == ST_OK && (pass == 0 ? solve : redo);
            if (!wave_any(act)) continue;
            const int qn = q + p;
            if (act && qlo == 0) {
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    int i = r * G + gl;
                    y[r] = (i < m && i == kidx) ? 1.0 : 0.0;
#pragma unroll
                    for (int c = 0; c < QMAX; ++c) b[r][c] = 0.0;
                }
            }
            const int qmaxw = wave_max_i(act ? qn : 0);
            // ---- gather columns [qlo, qn) of A(I, J) through LDS staging
            bool lookup_fail = false;
            for (int it = 0; wave_any(act && qlo + it * STAGE < qn); ++it) {
                const int c0 = qlo + it * STAGE;
                const bool ract = act && c0 < qn;
#pragma unroll
                for (int s = 0; s < STAGE; ++s)
#pragma unroll
                    for (int r = 0; r < RPL; ++r) S.stage[s * MMAX + r * G + gl] = 0.0;
                wave_sync();
                // first G entries of each staged column: all loads issued together
                int64_t ce1[STAGE], ce0[STAGE];
                int rw[STAGE];
                double vv[STAGE];
#pragma unroll
                for (int s = 0; s < STAGE; ++s) {
                    const int c = c0 + s;
                    ce0[s] = 0;
                    ce1[s] = 0;
                    if (ract && c < qn) {
                        ce0[s] = S.cb[c];
                        ce1[s] = ce0[s] + S.cl[c];
                    }
                }
#pragma unroll
                for (int s = 0; s < STAGE; ++s) {
                    const int64_t e = ce0[s] + gl;
                    rw[s] = -1;
                    vv[s] = 0.0;
                    if (e < ce1[s]) {
                        rw[s] = A.rowidx[e];
                        vv[s] = A.val[e];
                    }
                }
#pragma unroll
                for (int s = 0; s < STAGE; ++s) {
                    if (rw[s] >= 0) {
                        const int sl = hfind<C::LOGHSI>(S.hI, rw[s]);
                        const int li = sl >= 0 ? S.hIv[sl] : -1;
                        if (li >= 0 && li < MMAX) S.stage[s * MMAX + li] = vv[s];
                        else lookup_fail = true;
                    }
                    // entries beyond the first G (long columns)
                    for (int64_t e = ce0[s] + G + gl; e < ce1[s]; e += G) {
                        const int sl = hfind<C::LOGHSI>(S.hI, A.rowidx[e]);
                        const int li = sl >= 0 ? S.hIv[sl] : -1;
                        if (li >= 0 && li < MMAX) S.stage[s * MMAX + li] = A.val[e];
                        else lookup_fail = true;
                    }
                }
                wave_sync();
                if (ract) {
#pragma unroll
                    for (int c = 0; c < QMAX; ++c) {
                        if (c >= qmaxw) continue;
                        const int s = c - c0;
                        if (s >= 0 && s < STAGE && c < qn) {
#pragma unroll
                            for (int r = 0; r < RPL; ++r) {
                                b[r][c] = S.stage[s * MMAX + r * G + gl];
                            }
                        }
                    }
                }
                wave_sync();
            }
            if (lookup_fail) atomicOr(kargs()->err, 16);

            // ---- Householder QR update: stored reflectors j < qlo act on the new
            // columns only; reflectors qlo..qn-1 are formed and applied. In the larger
            // tiers, columns below the smallest qlo of the wave's solving groups are
            // final for every group: no reflector is formed there and no stored one is
            // applied to them (the first tier's blocks are too narrow for the test to
            // pay).
            const int qloww = QMAX > 12 ? -wave_max_i(act ? -qlo : -QMAX) : 0;
#pragma unroll
            for (int j = 0; j < QMAX; ++j) {
                if (j >= qmaxw) continue;
                const bool ja = act && j < qn;
                const bool newr = j >= qlo;
                double bj;
                // the reflector's vector: column j from its head row down, exact zeros
                // above it (the entries of R there), so that the products with the
                // other columns need no per-row predicate
                double vr[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) vr[r] = (r * G + gl >= j) ? b[r][j] : 0.0;
                if (j < qloww) {
                    bj = gsum<G>((gl == j % G) ? bt[j / G] : 0.0);
                } else {
                    double s2 = 0.0, x0p = 0.0;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) {
                        const int i = r * G + gl;
                        s2 += vr[r] * vr[r];
                        if (i == j) x0p = b[r][j];
                    }
                    s2 = gsum<G>(s2);
                    const double x0 = gsum<G>(x0p);
                    const double nx = sqrt(s2);
                    const double alpha = (x0 >= 0.0) ? -nx : nx;
                    const double vj = x0 - alpha;
                    const double bnew = (nx > 0.0) ? 1.0 / (nx * (nx + fabs(x0))) : 0.0;
                    if (ja && newr) {
                        if (!(nx > 0.0)) singular = true;
#pragma unroll
                        for (int r = 0; r < RPL; ++r)
                            if (r * G + gl == j) {
                                b[r][j] = vj;
                                vr[r] = vj;
                            }
#pragma unroll
                        for (int r = 0; r < RPL; ++r)
                            if (r * G + gl == j) {
                                rd[r] = alpha;
                                bt[r] = bnew;
                            }
                    }
                    double bold = 0.0;
                    if (wave_any(ja && !newr)) bold = gsum<G>((gl == j % G) ? bt[j / G] : 0.0);
                    bj = newr ? bnew : bold;
                }
                // the columns right of j in chunks of QCB: the chunk's products and
                // group sums are independent chains the wave issues interleaved
#pragma unroll
                for (int c0 = 0; c0 < QMAX; c0 += QCB) {
                    if (c0 + QCB - 1 <= j) continue;
                    if (c0 >= qmaxw || c0 + QCB <= qloww) continue;
                    double w[QCB];
#pragma unroll
                    for (int u = 0; u < QCB; ++u) {
                        const int c = c0 + u;
                        w[u] = 0.0;
                        if (c > j && c < QMAX) {
#pragma unroll
                            for (int r = 0; r < RPL; ++r) w[u] += vr[r] * b[r][c];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < QCB; ++u)
                        if (c0 + u > j && c0 + u < QMAX) w[u] = gsum<G>(w[u]);
#pragma unroll
                    for (int u = 0; u < QCB; ++u) {
                        const int c = c0 + u;
                        if (c > j && c < QMAX) {
                            const bool ca = ja && c < qn && (newr || c >= qlo);
                            if (ca) {
                                const double f = bj * w[u];
#pragma unroll
                                for (int r = 0; r < RPL; ++r) b[r][c] -= f * vr[r];
                            }
                        }
                    }
                }
                if (wave_any(ja && newr)) {
                    double w = 0.0;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) w += vr[r] * y[r];
                    w = gsum<G>(w);
                    if (ja && newr) {
                        const double f = bj * w;
#pragma unroll
                        for (int r = 0; r < RPL; ++r) y[r] -= f * vr[r];
                    }
                }
            }
            // ---- back substitution R m = (Q^T e)(0:qn)
            {
                double z[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) z[r] = y[r];
#pragma unroll
                for (int j = QMAX - 1; j >= 0; --j) {
                    if (j >= qmaxw) continue;
                    const bool ja = act && j < qn;
                    constexpr int dummy = 0;
                    (void)dummy;
                    const bool own = (gl == j % G);
                    double val = 0.0;
                    if (own && ja) val = z[j / G] / rd[j / G];
                    const double mj = gsum<G>(val);
                    if (ja) {
                        if (gl == 0) S.mt[j] = mj;
#pragma unroll
                        for (int r = 0; r < RPL; ++r)
                            if (r * G + gl < j) z[r] -= b[r][j] * mj;
                    }
                }
            }
            // ---- residual norm ||(Q^T e)(qn:m)||, plus r(k) = -1 if k is not in I
            {
                double s = 0.0;
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    const int i = r * G + gl;
                    if (i >= qn && i < m) s += y[r] * y[r];
                }
                s = gsum<G>(s);
                if (act) {
                    rn = sqrt(s + (kidx < 0 ? 1.0 : 0.0));
                    if (qmod >= 0) fl += solve_flops(mmod, m, qmod, qn);
                    q = qn;
                    p = 0;
                    if (singular) status = ST_SINGULAR;
                }
            }
            // ---- dropping (Section 4): after the pass-0 solve only
            if (pass == 0) {
                bool dact = act && dropok && P.drop != DROP_NONE && status == ST_OK;
                unsigned keep = 0u;
                if (dact) {
                    const double t = (P.drop == DROP_FIXED)
                                         ? P.tol
                                         : P.eps / ((double)q * __longlong_as_double((long long)*A.norm1_bits));
#pragma unroll
                    for (int c = 0; c < QMAX; ++c)
                        if (c < q && fabs(S.mt[c]) > t) keep |= 1u << c;
                    if (__popc(keep) == q) dact = false;
                }
                if (wave_any(dact)) {
                    int jv[(QMAX + G - 1) / G], lv[(QMAX + G - 1) / G];
                    int64_t bv0[(QMAX + G - 1) / G];
                    if (dact) {
                        if (keep == 0u) {
                            // keep the largest |m_j| (smaller column index on ties)
                            double bv = -1.0;
                            int bc = 0, bg = INT_MAX;
#pragma unroll
                            for (int c = 0; c < QMAX; ++c) {
                                if (c < q) {
                                    const double a = fabs(S.mt[c]);
                                    const int gj = S.Jlist[c];
                                    if (a > bv || (a == bv && gj < bg)) { bv = a; bc = c; bg = gj; }
                                }
                            }
                            keep = 1u << bc;
                        }
#pragma unroll
                        for (int s = 0; s < (QMAX + G - 1) / G; ++s) {
                            const int c = s * G + gl;
                            jv[s] = (c < q) ? S.Jlist[c] : 0;
                            bv0[s] = (c < q) ? S.cb[c] : 0;
                            lv[s] = (c < q) ? S.cl[c] : 0;
                        }
                    }
                    wave_sync();
                    if (dact) {
#pragma unroll
                        for (int s = 0; s < (QMAX + G - 1) / G; ++s) {
                            const int c = s * G + gl;
                            if (c < q && (keep & (1u << c))) {
                                const int d = __popc(keep & ((1u << c) - 1u));
                                S.Jlist[d] = jv[s];
                                S.cb[d] = bv0[s];
                                S.cl[d] = lv[s];
                            }
                        }
                        for (int t = gl; t < C::HSJ; t += G) S.hJ[t] = HEMPTY;
                    }
                    wave_sync();
                    if (dact) {
                        const int nk = __popc(keep);
                        for (int t = gl; t < nk; t += G) {
                            int sl;
                            hinsert<C::LOGHSJ>(S.hJ, S.Jlist[t], sl);
                        }
                        q = 0;
                        p = nk;
                        qlo = 0;
                        qmod = 0;
                        redo = true;
                    }
                    wave_sync();
                }
            }
        }

        // ============================================= I. stop test (step 3)
        bool finish = busy && (status != ST_OK || rn <= P.eps || l >= P.lmax);

        // ============================= J. dominant rows of the residual (step 4)
        const bool sel = busy && !finish;
        if (wave_any(sel)) {
            const int qmaxw = wave_max_i(sel ? q : 0);
            // r = A(I,J) m - e_k(I), eq. (2.4), formed from the sparse columns of A with
            // the columns taken in ascending global order. Rows whose coefficients tie
            // give bitwise-equal residuals, so exact ties reach the index tie-break.
            double *racc = S.racc();           // [MMAX] accumulator
            const double *mts = S.mt;          // [QMAX] solution values by slot
            int *ord = S.ord();                // [QMAX] slots in ascending column order
            if (sel) {
#pragma unroll
                for (int s = 0; s < (QMAX + G - 1) / G; ++s) {
                    const int c = s * G + gl;
                    if (c < q) {
                        const int jc = S.Jlist[c];
                        int rank = 0;
                        for (int t = 0; t < q; ++t) rank += (S.Jlist[t] < jc) ? 1 : 0;
                        ord[rank] = c;
                    }
                }
#pragma unroll
                for (int r = 0; r < RPL; ++r) racc[r * G + gl] = 0.0;
            }
            wave_sync();
            bool lookup_fail2 = false;
            // Fast path: when no column of the group has more than G entries, each lane
            // holds at most one entry per column, and the loads of all columns go out
            // together; the accumulation below keeps the ascending column order.
            bool shortcols = false;
            if constexpr (C::FASTSEL) {
                shortcols = true;
                int rw2[QMAX];
                double vv2[QMAX];
#pragma unroll
                for (int t = 0; t < QMAX; ++t) {
                    rw2[t] = -1;
                    vv2[t] = 0.0;
                    if (sel && t < q) {
                        const int64_t e0 = S.cb[ord[t]], e1 = e0 + S.cl[ord[t]];
                        if (e1 - e0 > G) shortcols = false;
                        const int64_t e = e0 + gl;
                        if (e < e1) {
                            rw2[t] = A.rowidx[e];
                            vv2[t] = A.val[e];
                        }
                    }
                }
                shortcols = gsum_i<G>(shortcols ? 0 : 1) == 0;
                if (sel && shortcols) {
#pragma unroll
                    for (int t = 0; t < QMAX; ++t) {
                        if (rw2[t] >= 0) {
                            const double mc = mts[ord[t]];
                            const int sl = hfind<C::LOGHSI>(S.hI, rw2[t]);
                            const int li = sl >= 0 ? S.hIv[sl] : -1;
                            if (li >= 0 && li < MMAX) racc[li] = __fma_rn(vv2[t], mc, racc[li]);
                            else lookup_fail2 = true;
                        }
                    }
                }
            }
            for (int t = 0; t < qmaxw; ++t) {
                if (sel && !shortcols && t < q) {
                    const int c = ord[t];
                    const double mc = mts[c];
                    const int64_t e1 = S.cb[c] + S.cl[c];
                    for (int64_t e = S.cb[c] + gl; e < e1; e += G) {
                        const int sl = hfind<C::LOGHSI>(S.hI, A.rowidx[e]);
                        const int li = sl >= 0 ? S.hIv[sl] : -1;
                        if (li >= 0 && li < MMAX) racc[li] = __fma_rn(A.val[e], mc, racc[li]);
                        else lookup_fail2 = true;
                    }
                }
                // rows of one column are distinct; successive columns are ordered by
                // the wave's in-order LDS execution
            }
            wave_sync();
            if (lookup_fail2) atomicOr(kargs()->err, 16);
            double ra[RPL];
            int gi[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = r * G + gl;
                const double ri = racc[i] - ((i == kidx) ? 1.0 : 0.0);
                const bool cand = sel && i < m && ri != 0.0 && !(rflag & (1u << r));
                ra[r] = cand ? fabs(ri) : -1.0;
                gi[r] = cand ? S.Ilist[i] : INT_MAX;
            }
            bool kcand = sel && kidx < 0 && !kR;  // r(k) = -1 when k is not in I
            unsigned chosen = 0u;
            int nsel = 0;
#pragma unroll
            for (int t = 0; t < CMAX; ++t) {
                if (t >= P.c) continue;
                double a = -1.0;
                int g = INT_MAX;
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    if (!(chosen & (1u << r)) && ra[r] >= 0.0 && (ra[r] > a || (ra[r] == a && gi[r] < g))) {
                        a = ra[r];
                        g = gi[r];
                    }
                }
                gargmax<G>(a, g);
                if (kcand && (1.0 > a || (1.0 == a && k < g))) { a = 1.0; g = k; }
                if (sel && a >= 0.0) {
                    if (gl == 0) S.Rh[t] = g;
                    nsel = t + 1;
                    if (kcand && g == k) {
                        kcand = false;
                        kR = true;
                    } else {
#pragma unroll
                        for (int r = 0; r < RPL; ++r)
                            if (gi[r] == g && ra[r] >= 0.0) chosen |= 1u << r;
                    }
                }
            }
            if (sel) {
                rflag |= chosen;
                nRh = nsel;
                if (nsel == 0) finish = true;  // no candidate row left: r = 0 (Section 3)
                linc = true;
                dropok = true;
                if (kargs()->one_loop && nsel > 0) park = true;
            }
        }

        // ================================================== output of a column
        if (finish) {
            const int64_t slot = kargs()->arena_base + ucol * (int64_t)QMAX;
            const int qq = (status == ST_OK) ? q : 0;
            // m_k with its rows in ascending order (rank of each entry in the group)
#pragma unroll
            for (int s = 0; s < (QMAX + G - 1) / G; ++s) {
                const int c = s * G + gl;
                if (c < qq) {
                    const int jc = S.Jlist[c];
                    int rank = 0;
                    for (int t = 0; t < qq; ++t) rank += (S.Jlist[t] < jc) ? 1 : 0;
                    kargs()->out.arenaJ[slot + rank] = jc;
                    kargs()->out.arenaV[slot + rank] = S.mt[c];
                }
            }
            if (gl == 0) {
                kargs()->out.off[ucol] = slot;
                kargs()->out.nJ[ucol] = qq;
                kargs()->out.nI[ucol] = m;
                kargs()->out.loops[ucol] = l;
                kargs()->out.status[ucol] = status;
                kargs()->out.resnorm[ucol] = rn;
                kargs()->out.flops[ucol] = fl;
            }
            // R of the final solve for the adjoint: row i of R is held by the owner lane
            // of row i (diagonal in rd, the rest in the block). Small tiers pack it in the
            // staging tile first, so the global stores need no per-entry addressing.
            if (kargs()->out.fac != nullptr) {
                const long long fo = fac_take(kargs()->out, fch, (gl == 0 && qq > 0) ? qq + qq * (qq + 1) / 2 : 0);
                if (gl == 0) {
                    kargs()->out.foff[ucol] = fo;
                    S.fo_lo = (int)(fo & 0xffffffffLL);
                    S.fo_hi = (int)(fo >> 32);
                }
                if constexpr (QMAX * (QMAX + 1) / 2 <= C::STAGE * MMAX) {
#pragma unroll
                    for (int r = 0; r < RPL; ++r) {
                        const int i = r * G + gl;
                        if (i < qq) {
                            const int base = (int)fac_row(qq, i) - qq;
                            S.stage[base] = rd[r];
#pragma unroll
                            for (int c = 0; c < QMAX; ++c)
                                if (c > i && c < qq) S.stage[base + c - i] = b[r][c];
                        }
                    }
                    wave_sync();
                    const long long fo = ((long long)S.fo_hi << 32) | (long long)(unsigned)S.fo_lo;
                    if (fo >= 0) {
                        double *F = kargs()->out.fac + fo;
                        const int tot = qq + qq * (qq + 1) / 2;
                        for (int t = gl; t < tot; t += G) F[t] = (t < qq) ? (double)S.Jlist[t] : S.stage[t - qq];
                    }
                } else {
                    wave_sync();
                    const long long fo = ((long long)S.fo_hi << 32) | (long long)(unsigned)S.fo_lo;
                    if (fo >= 0) {
                        double *F = kargs()->out.fac + fo;
                        for (int c = gl; c < qq; c += G) F[c] = (double)S.Jlist[c];
#pragma unroll
                        for (int r = 0; r < RPL; ++r) {
                            const int i = r * G + gl;
                            if (i < qq) {
                                double *Fr = F + fac_row(qq, i);
                                Fr[0] = rd[r];
#pragma unroll
                                for (int c = 0; c < QMAX; ++c)
                                    if (c > i && c < qq) Fr[c - i] = b[r][c];
                            }
                        }
                    }
                }
            }
            busy = false;
        }
        wave_sync();
    }
}

template <class C>
static void launch_tier(const TierArgs &a, int waves, hipStream_t s) {
    if (a.nmat > 1) hipLaunchKernelGGL((tier_kernel<C, true>), dim3(waves), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((tier_kernel<C, false>), dim3(waves), dim3(64), 0, s, a);
}

}  // namespace rsai
