// rorbk_api.hip -- host runtime of the MI355X ROR-BK library: argument
// checking, workspace management, the iteration driver (Algorithm 1), the
// FP32/BF16 + FP64 refinement loop, and the adjoint driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "rorbk_internal.h"

using namespace rorbk;

namespace {

thread_local char g_msg[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? RORBK_ERR_OOM : RORBK_ERR_HIP,        \
                        "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                        \
    } while (0)

#define CHK(expr)                \
    do {                         \
        int rc_ = (expr);        \
        if (rc_) return rc_;     \
    } while (0)

size_t dtype_size(int dt) { return dt == RORBK_F64 ? 8 : (dt == RORBK_F32 ? 4 : 2); }
size_t vec_size(int vec) { return vec == VEC_F64 ? 8 : 4; }

template <typename P>
int dalloc(P **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(P));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(RORBK_ERR_OOM, "hipMalloc of %zu bytes failed: %s", count * sizeof(P),
                    hipGetErrorString(e));
    }
    return RORBK_OK;
}

template <typename P>
void dfree(P *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

bool aligned16(const void *p, int64_t ld, size_t es) {
    return ((uintptr_t)p % 16 == 0) && ((ld * (int64_t)es) % 16 == 0);
}
// Blocks per selection chunk: whole blocks of at most 4096 rows (256 blocks).
// With many column segments, chunks of at most 8192 partial products (one
// workgroup sums a chunk's segments, bound by its own load rate, so more and
// smaller chunks finish sooner), as long as every chunk's candidate list
// still fits one merge workgroup (SEL_MERGE / K lists, K <= bmax).  Every
// chunk holds at least one whole block, hence at least K rows.
static int64_t sel_blocks_per_chunk(int64_t k, int64_t bmax, int64_t nseg) {
    int64_t bpc = 4096 / bmax;
    if (bpc > 256) bpc = 256;
    if (bpc < 1) bpc = 1;
    if (nseg > 2) {
        const int64_t per = 8192 / bmax;
        int64_t b2 = (8192 / nseg) / bmax;
        const int64_t bmin = (k + per - 1) / per;
        if (b2 < bmin) b2 = bmin;
        if (b2 < 1) b2 = 1;
        if (b2 < bpc) bpc = b2;
    }
    return bpc;
}


// Column chunking of the block step, the greedy Gram and the selection.
void plan_layout(Layout &L, bool col) {
    const int64_t n = L.n;
    const bool big = L.format == RORBK_DENSE && (L.bmax > RORBK_MAX_BLOCK_ROWS + 1 || col);
    if (big && col) {
        // column form: 128-column update slabs as for large blocks; the greedy
        // column Gram splits the K gathered rows into chunks (multiples of 16
        // rows) so that tiles x chunks is about 1024 workgroups
        L.wu = 128;
        L.nch_u = (int32_t)((n + 127) / 128);
        const int64_t nt = (n + 31) / 32, tiles = nt * (nt + 1) / 2;
        int64_t nch = (1024 + tiles - 1) / tiles;
        const int64_t maxch = (L.K + 15) / 16;
        if (nch > maxch) nch = maxch;
        if (nch < 1) nch = 1;
        int64_t wg = (L.K + nch - 1) / nch;
        wg = ((wg + 15) / 16) * 16;
        L.wg = wg;
        L.nch_g = (int32_t)((L.K + wg - 1) / wg);
        L.nseg = (int32_t)((n + 2047) / 2048);
    } else if (big) {
        // large blocks: one 128-column slab per update workgroup (row chunks
        // add the rest of the parallelism).  Greedy Gram on 32 x 32 tiles:
        // chunks sized so that tiles x chunks is about 1024 workgroups.  On
        // 64 x 64 tiles (one workgroup per CU at a time) the chunk count c
        // (up to 64, at least 256 columns each) minimises a time model in
        // microseconds: rounds of 256 workgroups times one workgroup's MFMA
        // time (n / c columns over 4 waves, 16 FP64 MFMAs of 64 cycles per 4
        // columns, 2.4 GHz), plus writing and reading c packed partials at
        // 5 TB/s
        L.wu = 128;
        L.nch_u = (int32_t)((n + 127) / 128);
        int64_t nch;
        if (gram64_for(L.dtype, L.K)) {
            const int64_t nt = (L.K + 63) / 64, tiles = nt * (nt + 1) / 2;
            const double kp = 0.5 * (double)L.K * (double)(L.K + 1);
            int64_t cap = n / 256;
            if (cap > 64) cap = 64;
            if (cap < 1) cap = 1;
            nch = 1;
            double best = 1e300;
            for (int64_t c = 1; c <= cap; ++c) {
                const double wg_us = (double)n / (double)c / 4.0 * 256.0 / 2400.0;
                const double cost = (double)((tiles * c + 255) / 256) * wg_us +
                                    (double)c * kp * 16.0 / 5.0e6;
                if (cost < best * (1.0 - 1e-9)) { best = cost; nch = c; }
            }
        } else {
            const int64_t nt = (L.K + 31) / 32, tiles = nt * (nt + 1) / 2;
            nch = (1024 + tiles - 1) / tiles;
            if (nch > 64) nch = 64;
        }
        if (nch > (n + 31) / 32) nch = (n + 31) / 32;
        if (nch < 1) nch = 1;
        int64_t wg = (n + nch - 1) / nch;
        wg = ((wg + 31) / 32) * 32;
        L.wg = wg;
        L.nch_g = (int32_t)((n + wg - 1) / wg);
        L.nseg = (int32_t)((n + 2047) / 2048);
    } else if (L.format == RORBK_DENSE) {
        // 128-column slabs per update workgroup: one up to 64 slabs, then two
        // (the next slab's rows load while one is reduced) or more, so that
        // there are at most about 256 workgroups whose partial products the
        // next step sums; at most 8 (x stays in LDS)
        const int64_t slabs = (n + 127) / 128;
        int64_t per = 1;
        if (slabs > 64) {
            per = (slabs + 255) / 256;
            if (per < 2) per = 2;
        }
        if (per > 8) per = 8;
        L.wu = 128 * per;
        L.nch_u = (int32_t)((n + L.wu - 1) / L.wu);
        // greedy Gram: about 256 columns per workgroup, at most 64 chunks
        int64_t nch = (n + 255) / 256;
        if (nch > 64) nch = 64;
        if (nch < 1) nch = 1;
        int64_t wg = (n + nch - 1) / nch;
        wg = ((wg + 31) / 32) * 32;
        L.wg = wg;
        L.nch_g = (int32_t)((n + wg - 1) / wg);
        L.nseg = (int32_t)((n + 2047) / 2048);
    } else {
        L.wu = n;
        L.nch_u = 1;
        L.wg = n;
        L.nch_g = 1;
        L.nseg = 1;
    }
    L.bpc = sel_blocks_per_chunk(L.k, L.bmax, L.nseg);
    L.nch_s = (int32_t)((L.k + L.bpc - 1) / L.bpc);
}

void free_solve_buffers(rorbk_handle_s *h) {
    dfree(h->d_tau);
    h->tau_cap = 0;
    dfree(h->d_recI);
    dfree(h->d_recR);
    h->rec_cap = 0;
    dfree(h->d_ckpt);
    h->ckpt_cap = 0;
    dfree(h->d_ckst);
    h->ckst_cap = 0;
}

void destroy_all(rorbk_handle_s *h) {
    dfree(h->d_off);
    dfree(h->d_S);
    dfree(h->d_pbar);
    dfree(h->d_W);
    dfree(h->d_hoff);
    dfree(h->d_H);
    dfree(h->d_ctrl);
    if (h->h_ctrl) (void)hipHostFree(h->h_ctrl);
    h->h_ctrl = nullptr;
    dfree(h->d_P[0]);
    dfree(h->d_P[1]);
    dfree(h->d_P3);
    dfree(h->d_XG);
    dfree(h->d_z3);
    dfree(h->d_fwdcnt);
    dfree(h->d_C);
    dfree(h->d_axp);
    dfree(h->d_r);
    dfree(h->d_bn);
    dfree(h->d_cn);
    dfree(h->d_ckey);
    dfree(h->d_cidx);
    dfree(h->d_ckey2);
    dfree(h->d_cidx2);
    dfree(h->d_I);
    dfree(h->d_rI);
    dfree(h->d_y);
    dfree(h->d_G);
    dfree(h->d_red);
    dfree(h->d_selcnt);
    dfree(h->d_ysum);
    dfree(h->d_ysum32);
    dfree(h->d_alg2);
    dfree(h->d_bigG);
    dfree(h->d_bigL);
    dfree(h->d_bigW);
    dfree(h->d_bigr);
    dfree(h->d_bigy);
    {
        char *p1 = (char *)h->d_xold, *p2 = (char *)h->d_dxp;
        dfree(p1);
        dfree(p2);
        h->d_xold = nullptr;
        h->d_dxp = nullptr;
    }
    dfree(h->d_rhs32);
    dfree(h->d_d32);
    dfree(h->d_r64);
    dfree(h->d_rep_tau);
    dfree(h->d_rep_I);
    free_solve_buffers(h);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (h->evr[i][j]) (void)hipEventDestroy(h->evr[i][j]);
}

// ----------------------------------------------------------- dispatch ----

hipError_t step(const rorbk_handle_s *h, const StepArgs &a) {
    if (h->big) return launch_step_big(h, a, h->stream);
    if (h->L.format == RORBK_CSR) return launch_step_csr(h, a, h->stream);
    return launch_step_dense(h, a, h->stream);
}

hipError_t residual(const rorbk_handle_s *h, const void *A, int dt, int aligned, int vec,
                    const void *x, double *axp) {
    if (h->L.format == RORBK_CSR) return launch_residual_csr(h, A, dt, vec, x, axp, h->stream);
    return launch_residual_dense(h, A, dt, aligned, vec, x, axp, h->stream);
}

hipError_t gram(const rorbk_handle_s *h, const void *A, int dt, int aligned, const int32_t *idx,
                int K, double *G) {
    (void)aligned;
    if (h->L.format == RORBK_CSR) return launch_gram_csr(h, A, dt, idx, K, G, h->stream);
    if (K > RORBK_MAX_BLOCK_ROWS + 1) return launch_gram_big(h, A, dt, idx, K, G, h->stream);
    return launch_gram_dense(h, A, dt, idx, K, G, h->stream);
}

// Per-solve buffers sized by the iteration count.
int ensure_solve_buffers(rorbk_handle_s *h, int64_t iters, bool record_I, int64_t ckpt_slots,
                         int vec) {
    const Layout &L = h->L;
    if (h->tau_cap < iters) {
        dfree(h->d_tau);
        CHK(dalloc(&h->d_tau, (size_t)(3 * iters)));
        h->tau_cap = iters;
    }
    if (h->rec_cap < iters || (record_I && !h->d_recI)) {
        dfree(h->d_recI);
        dfree(h->d_recR);
        CHK(dalloc(&h->d_recR, (size_t)iters));
        if (record_I) CHK(dalloc(&h->d_recI, (size_t)(iters * L.K)));
        h->rec_cap = iters;
    }
    if (ckpt_slots > 0) {
        const int64_t need = ckpt_slots * L.n * (int64_t)vec_size(vec);
        if (h->ckpt_cap < need) {
            dfree(h->d_ckpt);
            CHK(dalloc((char **)&h->d_ckpt, (size_t)need));
            h->ckpt_cap = need;
        }
        if (h->chain && h->ckst_cap < ckpt_slots) {
            dfree(h->d_ckst);
            CHK(dalloc(&h->d_ckst, (size_t)(ckpt_slots * CKST_DOUBLES)));
            h->ckst_cap = ckpt_slots;
        }
    }
    return RORBK_OK;
}

struct RunOpts {
    int vec;
    const void *A;
    int dt;
    int aligned;
    const void *b;
    void *x;
    bool record_I;
    const int32_t *replay_I;   // device, indexed by iteration
    int64_t ckpt_every;        // 0: none
    void *ckpt;                // checkpoint slots (vector type)
    bool resume_chain;         // chain form: the sampled steps of it0 are done
                               // (restored from a checkpoint's chain state)
};

// Iterations [it0, it1) of Algorithm 1 on the device; stops early once the
// control block's done flag is set.  Returns the number of iterations whose
// residual was measured (the stopping one included).
int run_iterations(rorbk_handle_s *h, const RunOpts &o, int64_t it0, int64_t it1,
                   int64_t *ran, bool *stopped) {
    const Layout &L = h->L;
    hipStream_t s = h->stream;
    const bool fused = h->fast3 != 0;
    int ping = 0;
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.A = o.A;
    a.dt = o.dt;
    a.aligned = o.aligned;
    a.vec = o.vec;
    a.b = o.b;
    a.x = o.x;
    a.gb = nullptr;
    FwdArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.A = o.A;
    fa.dt = o.dt;
    fa.aligned = o.aligned;
    fa.vec = o.vec;
    fa.b = o.b;
    fa.x = o.x;
    const int64_t xgs = 3 * L.bmax * L.bmax;   // one slot of cross-Grams
    // chain form: iteration it ends with the greedy update and the sampled
    // steps of it + 1 in one pass, unless it + 1 is the end.  A checkpoint at
    // it + 1 then keeps the state that pass starts from (x before it, the
    // greedy rows, y and the next z), from which the recomputation resumes
    // with the same arithmetic.
    const bool chain = fused && h->chain != 0;
    auto chain_next = [&](int64_t it) -> bool { return chain && it + 1 < it1; };
    bool prev_chained = chain && o.resume_chain;
    if (prev_chained) {
        // the caller restored x, I, y, z and ran the sampled steps of it0
    } else if (fused) {
        // the first iteration's three-block products and cross-Grams
        fa.I = nullptr;
        fa.tau_index = 3 * it0;
        HIPCHK(launch_fwd_greedy(h, fa, s));
        HIPCHK(launch_xgram(h, o.A, o.dt, o.aligned, 3 * it0, h->d_XG + (it0 & 1) * xgs, 4, s));
    } else {
        // partial products of the first sampled step
        a.cur.kind = -1;
        a.ymode = 2;
        a.nxt.kind = 0;
        a.nxt.tau_index = 3 * it0;
        a.Pout = h->d_P[ping ^ 1];
        HIPCHK(step(h, a));
        ping ^= 1;
    }

    const int64_t poll = 16;
    // residual-pass timings (iteration, ms); launches after the stopping
    // iteration return at once and are left out when the solve ends
    int timed_slot[2] = {0, 0};
    int64_t timed_it[2] = {0, 0};
    std::vector<std::pair<int64_t, float>> timings;
    auto take_time = [&](int slot) -> int {
        if (!timed_slot[slot]) return RORBK_OK;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->evr[slot][0], h->evr[slot][1]));
        timings.emplace_back(timed_it[slot], ms);
        timed_slot[slot] = 0;
        return RORBK_OK;
    };
    Ctrl *slots = h->h_ctrl + 1;  // two pinned slots after the mirror
    hipEvent_t evs[2] = {h->ev0, h->ev1};
    int64_t chunk = 0;
    bool done = false;
    for (int64_t it = it0; it < it1; ++it) {
        if (o.ckpt_every > 0 && (it % o.ckpt_every) == 0 && !prev_chained) {
            char *dst = (char *)o.ckpt + (size_t)(it / o.ckpt_every) * L.n * vec_size(o.vec);
            HIPCHK(hipMemcpyAsync(dst, o.x, (size_t)L.n * vec_size(o.vec),
                                  hipMemcpyDeviceToDevice, s));
        }
        if (fused) {
            if (!prev_chained) {
                fa.I = nullptr;
                fa.y = nullptr;
                fa.tau_index = 3 * it;
                fa.xg = h->d_XG + (it & 1) * xgs;
                HIPCHK(launch_fwd_samp3(h, fa, s));
            }
        } else {
            for (int l = 0; l < 3; ++l) {
                a.cur.kind = 0;
                a.cur.tau_index = 3 * it + l;
                a.ymode = 0;
                a.Pin = h->d_P[ping];
                if (l < 2) {
                    a.nxt.kind = 0;
                    a.nxt.tau_index = 3 * it + l + 1;
                    a.Pout = h->d_P[ping ^ 1];
                } else {
                    a.nxt.kind = -1;
                    a.Pout = nullptr;
                }
                HIPCHK(step(h, a));
                if (l < 2) ping ^= 1;
            }
        }
        const bool timed = h->profile && ((it - it0) % poll) == 0;
        if (timed) HIPCHK(hipEventRecord(h->evr[chunk & 1][0], s));
        if (fused) {
            // the next iteration's cross-Grams ride along in spare workgroups
            // (the chain form forms them after the selection)
            XgSide side = {h->d_tau, 3 * (it + 1), L.q, L.rem, (int)L.bmax, 0,
                           h->d_XG + ((it + 1) & 1) * xgs};
            if (it + 1 < it1 && !chain) side.jobs = fwd_xgram_jobs((int)L.bmax);
            HIPCHK(launch_residual_dense_side(h, o.A, o.dt, o.aligned, o.vec, o.x, h->d_axp, side,
                                              s));
        } else {
            HIPCHK(residual(h, o.A, o.dt, o.aligned, o.vec, o.x, h->d_axp));
        }
        if (timed) {
            HIPCHK(hipEventRecord(h->evr[chunk & 1][1], s));
            timed_slot[chunk & 1] = 1;
            timed_it[chunk & 1] = it;
        }
        SelectArgs sa;
        memset(&sa, 0, sizeof(sa));
        sa.vec = o.vec;
        sa.b = o.b;
        sa.axp = h->d_axp;
        sa.nseg = L.nseg;
        sa.r = h->d_r;
        sa.it = it;
        sa.record_rrn = 1;
        sa.rec_rrn = h->d_recR;
        sa.record_I = o.record_I ? 1 : 0;
        sa.rec_I = h->d_recI;
        sa.replay_I = o.replay_I;
        sa.I_out = h->d_I;
        sa.rI_out = h->d_rI;
        sa.stop_test = 1;
        sa.skip_topk = 0;
        if (chain_next(it)) {
            // the next iteration's cross-Grams in the selection's spare workgroups
            sa.xg_out = h->d_XG + ((it + 1) & 1) * xgs;
            sa.xg_A = o.A;
            sa.xg_dt = o.dt;
            sa.xg_aligned = o.aligned;
            sa.xg_ti = 3 * (it + 1);
        }
        HIPCHK(launch_select(h, sa, s));
        if (chain_next(it)) {
            // greedy Gram and C; y and the next z; the greedy update with the
            // next iteration's sampled steps
            double *xgn = h->d_XG + ((it + 1) & 1) * xgs;
            HIPCHK(launch_gram_chain(h, o.A, o.dt, o.aligned, h->d_I, 3 * (it + 1), h->d_G, s));
            double *ckst = nullptr;
            if (o.ckpt_every > 0 && ((it + 1) % o.ckpt_every) == 0) {
                const int64_t slot = (it + 1) / o.ckpt_every;
                char *dst = (char *)o.ckpt + (size_t)slot * L.n * vec_size(o.vec);
                HIPCHK(hipMemcpyAsync(dst, o.x, (size_t)L.n * vec_size(o.vec),
                                      hipMemcpyDeviceToDevice, s));
                ckst = h->d_ckst + slot * CKST_DOUBLES;
            }
            fa.I = h->d_I;
            fa.y = h->d_y;
            fa.tau_index = 3 * (it + 1);
            fa.xg = xgn;
            HIPCHK(launch_fwd_chain(h, fa, h->d_r, ckst, s));
            prev_chained = true;
        } else if (h->col) {
            HIPCHK(launch_col_greedy(h, o.A, o.dt, o.aligned, o.vec, o.x, h->d_I, (int)L.K,
                                     h->d_rI, h->d_y, s));
        } else {
            HIPCHK(gram(h, o.A, o.dt, o.aligned, h->d_I, (int)L.K, h->d_G));
            HIPCHK(launch_chol_solve(h, h->d_G, (int)L.K, h->d_rI, nullptr, h->d_y, s));
        }
        if (chain_next(it)) {
            // done above
        } else if (fused) {
            // greedy update and the next iteration's three-block products
            fa.I = h->d_I;
            fa.y = h->d_y;
            fa.tau_index = (it + 1 < it1) ? 3 * (it + 1) : -1;
            HIPCHK(launch_fwd_greedy(h, fa, s));
            prev_chained = false;
        } else {
            a.cur.kind = 1;
            a.cur.count = (int32_t)L.K;
            a.cur.idx = h->d_I;
            a.ymode = 1;
            a.ygiven = h->d_y;
            if (it + 1 < it1) {
                a.nxt.kind = 0;
                a.nxt.tau_index = 3 * (it + 1);
                a.Pout = h->d_P[ping ^ 1];
            } else {
                a.nxt.kind = -1;
                a.Pout = nullptr;
            }
            HIPCHK(step(h, a));
            if (it + 1 < it1) ping ^= 1;
        }
        // poll the stop flag one chunk behind so the device never starves
        if (((it + 1 - it0) % poll) == 0 && it + 1 < it1) {
            const int slot = (int)(chunk & 1);
            HIPCHK(hipMemcpyAsync(&slots[slot], h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(evs[slot], s));
            if (chunk > 0) {
                const int prev = slot ^ 1;
                HIPCHK(hipEventSynchronize(evs[prev]));
                if (slots[prev].done) done = true;
                CHK(take_time(prev));
            }
            ++chunk;
            if (done) break;
        }
    }
    HIPCHK(hipMemcpyAsync(h->h_ctrl, h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    CHK(take_time(0));
    CHK(take_time(1));
    const Ctrl &c = *h->h_ctrl;
    if (c.status != RORBK_OK)
        return fail(c.status, c.status == RORBK_ERR_NONFINITE
                                  ? "non-finite residual at iteration %lld"
                                  : "block Gram not positive definite at iteration %lld",
                    (long long)c.last_it);
    for (const auto &tm : timings)
        if (!c.done || tm.first <= c.conv_it) {
            h->prof_in_ms += tm.second;
            h->prof_in_n += 1;
        }
    if (c.done) {
        *ran = c.conv_it - it0 + 1;
        *stopped = true;
    } else {
        *ran = it1 - it0;
        *stopped = false;
    }
    return RORBK_OK;
}

// The selections (tau) of iterations [0, iters) of a solve starting at
// start_iter: sampled on the device, or copied from the replay table.
int prepare_tau(rorbk_handle_s *h, uint64_t seed, int64_t start_iter, int64_t iters, bool replay) {
    if (replay)
        HIPCHK(launch_copy_tau(h->d_rep_tau, h->d_tau, 3 * iters, h->stream));
    else
        HIPCHK(launch_sample(seed, start_iter, iters, h->d_W, h->L.k, h->d_tau, h->stream));
    return RORBK_OK;
}

}  // namespace

// ======================================================================= ABI

extern "C" {

const char *ror_bk_error_string(int code) {
    switch (code) {
    case RORBK_OK: return "ok";
    case RORBK_ERR_INVALID_ARG: return "invalid argument";
    case RORBK_ERR_OOM: return "out of memory";
    case RORBK_ERR_HIP: return "HIP runtime error";
    case RORBK_ERR_NOT_SPD: return "block Gram not positive definite";
    case RORBK_ERR_NONFINITE: return "non-finite residual";
    case RORBK_ERR_NOT_RECORDED: return "no recorded solve for backward";
    case RORBK_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}

const char *ror_bk_last_error_message(void) { return g_msg; }

int ror_bk_destroy(rorbk_handle h) {
    if (!h) return RORBK_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    destroy_all(h);
    delete h;
    return RORBK_OK;
}

int ror_bk_partition(int64_t m, int64_t block_rows, int64_t *offsets_host, int64_t *k) {
    g_msg[0] = 0;
    if (!k) return fail(RORBK_ERR_INVALID_ARG, "k pointer is NULL");
    if (m < 1) return fail(RORBK_ERR_INVALID_ARG, "m = %lld < 1", (long long)m);
    if (block_rows < 1 || block_rows > m)
        return fail(RORBK_ERR_INVALID_ARG, "block_rows %lld outside [1, m=%lld]",
                    (long long)block_rows, (long long)m);
    const int64_t nb = m / block_rows, q = m / nb, rem = m - nb * q;
    *k = nb;
    if (offsets_host)
        for (int64_t t = 0; t <= nb; ++t) offsets_host[t] = t * q + std::min(t, rem);
    return RORBK_OK;
}

int ror_bk_setup(const rorbk_matrix *A, int64_t block_rows, double lambda, void *stream,
                 rorbk_handle *out) {
    g_msg[0] = 0;
    const auto t_entry = std::chrono::steady_clock::now();
    if (!out) return fail(RORBK_ERR_INVALID_ARG, "out handle pointer is NULL");
    *out = nullptr;
    if (!A) return fail(RORBK_ERR_INVALID_ARG, "matrix descriptor is NULL");
    if (A->format != RORBK_DENSE && A->format != RORBK_CSR)
        return fail(RORBK_ERR_INVALID_ARG, "unknown format %d", A->format);
    if (A->dtype != RORBK_F64 && A->dtype != RORBK_F32 && A->dtype != RORBK_BF16)
        return fail(RORBK_ERR_INVALID_ARG, "unknown dtype %d", A->dtype);
    if (A->m < 1 || A->n < 1) return fail(RORBK_ERR_INVALID_ARG, "empty matrix %lld x %lld",
                                          (long long)A->m, (long long)A->n);
    if (A->m > INT32_MAX || A->n > INT32_MAX)
        return fail(RORBK_ERR_UNSUPPORTED, "dimensions above 2^31 are not supported");
    if (!A->values && !(A->format == RORBK_CSR && A->nnz == 0))
        return fail(RORBK_ERR_INVALID_ARG, "matrix values pointer is NULL");
    if (A->format == RORBK_DENSE && A->ld < A->n)
        return fail(RORBK_ERR_INVALID_ARG, "ld %lld < n %lld", (long long)A->ld, (long long)A->n);
    if (A->format == RORBK_CSR) {
        if (!A->rowptr || A->nnz < 0)
            return fail(RORBK_ERR_INVALID_ARG, "CSR needs rowptr and nnz >= 0");
        if (A->dtype == RORBK_BF16)
            return fail(RORBK_ERR_UNSUPPORTED, "BF16 storage is dense only");
        if (A->nnz > 0 && (!A->colidx || !A->values))
            return fail(RORBK_ERR_INVALID_ARG, "CSR with nnz > 0 needs colidx and values");
    }
    if (block_rows < 1 || block_rows > A->m)
        return fail(RORBK_ERR_INVALID_ARG, "block_rows %lld outside [1, m=%lld]",
                    (long long)block_rows, (long long)A->m);
    if (!(lambda >= 0.0) || !std::isfinite(lambda))
        return fail(RORBK_ERR_INVALID_ARG, "lambda must be finite and >= 0");

    rorbk_handle_s *h = new (std::nothrow) rorbk_handle_s;
    if (!h) return fail(RORBK_ERR_OOM, "host allocation failed");
    memset(h, 0, sizeof(*h));
    Layout &L = h->L;
    L.m = A->m;
    L.n = A->n;
    L.ld = A->format == RORBK_DENSE ? A->ld : A->n;
    L.nnz = A->nnz;
    L.format = A->format;
    L.dtype = A->dtype;
    L.k = A->m / block_rows;
    L.q = A->m / L.k;
    L.rem = A->m - L.k * L.q;
    L.K = L.q;
    L.bmax = L.q + (L.rem > 0 ? 1 : 0);
    if (L.bmax > RORBK_MAX_BLOCK_ROWS + 1) {
        const int lim = (L.format == RORBK_DENSE) ? RORBK_MAX_BIG_BLOCK_ROWS
                                                  : RORBK_MAX_BLOCK_ROWS + 1;
        if (L.bmax > lim) {
            delete h;
            return fail(RORBK_ERR_UNSUPPORTED, "blocks of %lld rows exceed the supported %d%s",
                        (long long)L.bmax, lim,
                        L.format == RORBK_DENSE ? "" : " for CSR storage");
        }
        h->big = 1;
    }
    // column form (Sec. 3.1): blocks with at least as many rows as columns, in
    // the large-block regime (smaller blocks keep the row form, whose systems
    // are at most RORBK_MAX_BLOCK_ROWS + 1 square)
    if (h->big && L.q >= L.n) h->col = 1;
    plan_layout(L, h->col != 0);
    h->stream = (hipStream_t)stream;
    h->lambda = lambda;
    h->A = A->values;
    h->A64 = (A->dtype == RORBK_F64) ? (const double *)A->values : A->values_f64;
    h->rowptr = A->rowptr;
    h->colidx = A->colidx;
    const bool dense = A->format == RORBK_DENSE;
    h->aligned = (dense && aligned16(A->values, L.ld, dtype_size(A->dtype))) ? 1 : 0;
    h->aligned64 = (dense && h->A64 && aligned16(h->A64, L.ld, 8)) ? 1 : 0;
    h->refine_inner = 50;
    h->refine_eta = 1e-4;
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            ncu <= 0)
            ncu = 256;
        h->ncu = ncu;
    }

    const int64_t k = L.k, K = L.K, bmax = L.bmax;
    const int64_t q = L.q, rem = L.rem;
    const int64_t htotal = h->col ? k * L.n * L.n : rem * (q + 1) * (q + 1) + (k - rem) * q * q;
    const int64_t gdim = h->col ? L.n : K;   // size of the greedy system
    int rc = RORBK_OK;
#define ALLOC(p, n)                                   \
    do {                                              \
        rc = dalloc(&(p), (size_t)(n));               \
        if (rc) { destroy_all(h); delete h; return rc; } \
    } while (0)
    ALLOC(h->d_off, k + 1);
    ALLOC(h->d_hoff, k + 1);
    ALLOC(h->d_S, k);
    ALLOC(h->d_pbar, k);
    ALLOC(h->d_W, k);
    ALLOC(h->d_H, htotal);
    ALLOC(h->d_ctrl, 1);
    ALLOC(h->d_P[0], (int64_t)L.nch_u * bmax);
    ALLOC(h->d_P[1], (int64_t)L.nch_u * bmax);
    // dense row-form blocks of at most RORBK_FWD_MAX_BLOCK rows: fused forward
    // steps (three-block partial products, two slots of cross-Grams)
    // (only where the chain form applies: with many columns the fused steps'
    // cross-Gram tiles over whole rows cost more than the separate steps)
    h->fast3 = (L.format == RORBK_DENSE && !h->big && !h->col &&
                bmax <= RORBK_FWD_MAX_BLOCK && L.K <= 64 && L.n <= 4096 &&
                L.nch_s * L.K <= 8192) ? 1 : 0;
    if (h->fast3) {
        // column slabs of the fused steps: sub-slabs of 64 (FP64 storage) or
        // 128 columns; one per workgroup up to 64 of them, else several, for
        // at most about 256 workgroups (x of a slab stays in LDS: <= 1024)
        const int64_t swc = (L.dtype == RORBK_F64) ? 64 : 128;
        const int64_t slabs = (L.n + swc - 1) / swc;
        int64_t per = 1;
        if (slabs > 64) {
            per = (slabs + 255) / 256;
            if (per < 2) per = 2;
        }
        if (per > 1024 / swc) per = 1024 / swc;
        L.wf = per * swc;
        L.nch_f = (int32_t)((L.n + L.wf - 1) / L.wf);
        ALLOC(h->d_P3, (int64_t)L.nch_f * 3 * bmax);
        ALLOC(h->d_XG, 2 * 3 * bmax * bmax);
        ALLOC(h->d_z3, 3 * RORBK_FWD_MAX_BLOCK);
        ALLOC(h->d_fwdcnt, 1);
        // chain form: greedy sets of at most 64 rows, rows of at most 4096
        // columns (Grams after the selection in up to 4 column chunks of at
        // least 512) and a selection that merges its candidates in one level
        h->chain = (L.K <= 64 && L.n <= 4096 && L.nch_s * L.K <= 8192) ? 1 : 0;
        if (h->chain) {
            int64_t nc = (L.n + 511) / 512;
            if (nc > 4) nc = 4;
            int64_t wc = (L.n + nc - 1) / nc;
            wc = ((wc + 31) / 32) * 32;
            L.wc = wc;
            L.nch_c = (int32_t)((L.n + wc - 1) / wc);
            ALLOC(h->d_C, (int64_t)L.nch_c * 3 * RORBK_FWD_MAX_BLOCK * 64);
        }
    }
    ALLOC(h->d_axp, (int64_t)L.nseg * L.m);
    {
        char *r = nullptr;
        rc = dalloc(&r, (size_t)(8 * L.m));
        if (rc) { destroy_all(h); delete h; return rc; }
        h->d_r = r;
        char *r64 = nullptr;
        rc = dalloc(&r64, (size_t)(8 * L.m));
        if (rc) { destroy_all(h); delete h; return rc; }
        h->d_r64 = (double *)r64;
    }
    ALLOC(h->d_bn, k);
    ALLOC(h->d_cn, L.nch_s);
    ALLOC(h->d_ckey, (int64_t)L.nch_s * K);
    ALLOC(h->d_cidx, (int64_t)L.nch_s * K);
    ALLOC(h->d_ckey2, (int64_t)L.nch_s * K);
    ALLOC(h->d_cidx2, (int64_t)L.nch_s * K);
    ALLOC(h->d_I, bmax);
    ALLOC(h->d_rI, bmax);
    ALLOC(h->d_y, bmax);
    ALLOC(h->d_G, (int64_t)L.nch_g * gdim * (gdim + 1) / 2);
    ALLOC(h->d_red, 64);
    ALLOC(h->d_selcnt, 1);
    ALLOC(h->d_ysum, L.n);
    ALLOC(h->d_alg2, 3);
    if (h->big || gdim > 64) {
        // the blocked Cholesky of the greedy system (every greedy set of more
        // than 64 rows)
        const int64_t P = (gdim + 31) / 32;
        ALLOC(h->d_bigG, (P + 1) * 32 * P * 32);
        ALLOC(h->d_bigL, (P + 1) * 32 * P * 32);
        ALLOC(h->d_bigW, P * 32 * 32);
    }
    if (h->big) {
        ALLOC(h->d_bigr, bmax);
        ALLOC(h->d_bigy, bmax);
        char *p1 = nullptr, *p2 = nullptr;
        rc = dalloc(&p1, (size_t)(8 * L.n));
        if (rc) { destroy_all(h); delete h; return rc; }
        h->d_xold = p1;
        rc = dalloc(&p2, (size_t)(8 * L.n * ((bmax + 63) / 64)));
        if (rc) { destroy_all(h); delete h; return rc; }
        h->d_dxp = p2;
    }
#undef ALLOC
    hipError_t e = hipHostMalloc((void **)&h->h_ctrl, 3 * sizeof(Ctrl), hipHostMallocDefault);
    if (e != hipSuccess) {
        destroy_all(h);
        delete h;
        return fail(RORBK_ERR_OOM, "pinned allocation failed: %s", hipGetErrorString(e));
    }
    memset(h->h_ctrl, 0, 3 * sizeof(Ctrl));
    if (hipMemsetAsync(h->d_selcnt, 0, sizeof(uint32_t), (hipStream_t)stream) != hipSuccess ||
        (h->d_fwdcnt &&
         hipMemsetAsync(h->d_fwdcnt, 0, sizeof(uint32_t), (hipStream_t)stream) != hipSuccess)) {
        destroy_all(h);
        delete h;
        return fail(RORBK_ERR_HIP, "clearing the selection counter failed");
    }
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
        hipEventCreate(&h->evr[0][0]) != hipSuccess || hipEventCreate(&h->evr[0][1]) != hipSuccess ||
        hipEventCreate(&h->evr[1][0]) != hipSuccess || hipEventCreate(&h->evr[1][1]) != hipSuccess) {
        destroy_all(h);
        delete h;
        return fail(RORBK_ERR_HIP, "event creation failed");
    }

    auto bail = [&](int code) {
        destroy_all(h);
        delete h;
        return code;
    };
    hipStream_t s = h->stream;
    if (L.format == RORBK_CSR) {
        int32_t *d_bad = nullptr;
        rc = dalloc(&d_bad, 1);
        if (rc) return bail(rc);
        int32_t zero = 0, hbad = 0;
        hipError_t e1 = hipMemcpyAsync(d_bad, &zero, 4, hipMemcpyHostToDevice, s);
        hipError_t e2 = launch_csr_check(h, d_bad, s);
        hipError_t e3 = hipMemcpyAsync(&hbad, d_bad, 4, hipMemcpyDeviceToHost, s);
        hipError_t e4 = hipStreamSynchronize(s);
        dfree(d_bad);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess)
            return bail(fail(RORBK_ERR_HIP, "CSR check failed: %s",
                             hipGetErrorString(e2 != hipSuccess ? e2 : e4)));
        if (hbad)
            return bail(fail(RORBK_ERR_INVALID_ARG,
                             "CSR arrays invalid (rowptr not monotone from 0 to nnz, or column "
                             "indices not strictly ascending in [0, n) within a row)"));
    }
    if (launch_partition(L.m, k, h->d_off, h->d_hoff, s) != hipSuccess)
        return bail(fail(RORBK_ERR_HIP, "partition launch failed"));
    // centroid cosines and the proposal
    {
        const int64_t len = setup_proposal_scratch(k, L.n, h->ncu);
        double *scratch = nullptr;
        rc = dalloc(&scratch, (size_t)len);
        if (rc) return bail(rc);
        hipError_t le = (L.format == RORBK_CSR)
                            ? launch_setup_proposal_csr(h, h->A, L.dtype, scratch, s)
                            : launch_setup_proposal_dense(h, h->A, L.dtype, h->aligned, scratch, s);
        hipError_t se = hipStreamSynchronize(s);
        dfree(scratch);
        if (le != hipSuccess || se != hipSuccess)
            return bail(fail(RORBK_ERR_HIP, "proposal setup failed: %s",
                             hipGetErrorString(le != hipSuccess ? le : se)));
    }
    // stored block inverses
    {
        int32_t *d_fail = nullptr;
        rc = dalloc(&d_fail, 1);
        if (rc) return bail(rc);
        int32_t zero = 0, hfail = 0;
        hipError_t e1 = hipMemcpyAsync(d_fail, &zero, 4, hipMemcpyHostToDevice, s);
        hipError_t e2 = (L.format == RORBK_CSR)
                            ? launch_block_inverses_csr(h, h->A, L.dtype, d_fail, s)
                            : (h->col ? launch_col_block_inverses(h, h->A, L.dtype, d_fail, s)
                                      : launch_block_inverses_dense(h, h->A, L.dtype, h->aligned,
                                                                    d_fail, s));
        hipError_t e3 = hipMemcpyAsync(&hfail, d_fail, 4, hipMemcpyDeviceToHost, s);
        hipError_t e4 = hipStreamSynchronize(s);
        dfree(d_fail);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess)
            return bail(fail(RORBK_ERR_HIP, "block inverse setup failed: %s",
                             hipGetErrorString(e2 != hipSuccess ? e2 : e4)));
        if (hfail)
            return bail(fail(RORBK_ERR_NOT_SPD, h->col
                             ? "a block Gram A_t^T A_t + lambda I is not positive definite"
                             : "a block Gram A_t A_t^T + lambda I is not positive definite"));
    }
    h->t_setup_s =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_entry).count();
    *out = h;
    return RORBK_OK;
}

int ror_bk_get_sizes(rorbk_handle h, int64_t *k, int64_t *K, int64_t *bmax) {
    if (!h) return fail(RORBK_ERR_INVALID_ARG, "NULL handle");
    if (k) *k = h->L.k;
    if (K) *K = h->L.K;
    if (bmax) *bmax = h->L.bmax;
    return RORBK_OK;
}

int ror_bk_get_setup(rorbk_handle h, int64_t *offsets_host, double *S_host, double *pbar_host,
                     double *W_host) {
    if (!h) return fail(RORBK_ERR_INVALID_ARG, "NULL handle");
    const int64_t k = h->L.k;
    if (offsets_host)
        HIPCHK(hipMemcpyAsync(offsets_host, h->d_off, 8 * (k + 1), hipMemcpyDeviceToHost, h->stream));
    if (S_host) HIPCHK(hipMemcpyAsync(S_host, h->d_S, 8 * k, hipMemcpyDeviceToHost, h->stream));
    if (pbar_host)
        HIPCHK(hipMemcpyAsync(pbar_host, h->d_pbar, 8 * k, hipMemcpyDeviceToHost, h->stream));
    if (W_host) HIPCHK(hipMemcpyAsync(W_host, h->d_W, 8 * k, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RORBK_OK;
}

int ror_bk_set_proposal(rorbk_handle h, const double *W_host) {
    if (!h || !W_host) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    for (int64_t t = 0; t < h->L.k; ++t)
        if (!std::isfinite(W_host[t]) || W_host[t] < 0.0 || (t > 0 && W_host[t] < W_host[t - 1]))
            return fail(RORBK_ERR_INVALID_ARG, "W must be finite, non-negative, non-decreasing");
    HIPCHK(hipMemcpyAsync(h->d_W, W_host, 8 * h->L.k, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RORBK_OK;
}

int ror_bk_get_form(rorbk_handle h, int32_t *column_form) {
    if (!h || !column_form) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    *column_form = h->col;
    return RORBK_OK;
}

int ror_bk_get_block_inverse(rorbk_handle h, int64_t t, double *Hinv_host) {
    if (!h || !Hinv_host) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    const Layout &L = h->L;
    if (t < 0 || t >= L.k) return fail(RORBK_ERR_INVALID_ARG, "block %lld out of range", (long long)t);
    const int64_t big = std::min(t, L.rem);
    int64_t off = big * (L.q + 1) * (L.q + 1) + (t - big) * L.q * L.q;
    int64_t bt = L.q + (t < L.rem ? 1 : 0);
    if (h->col) {   // column form: (A_t^T A_t + lambda I)^{-1}, n x n
        off = t * L.n * L.n;
        bt = L.n;
    }
    HIPCHK(hipMemcpyAsync(Hinv_host, h->d_H + off, 8 * bt * bt, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RORBK_OK;
}

int ror_bk_sample(rorbk_handle h, uint64_t seed, int64_t j0, int64_t count, int32_t *tau_host) {
    if (!h || !tau_host || count < 0 || j0 < 0)
        return fail(RORBK_ERR_INVALID_ARG, "bad sample arguments");
    if (count == 0) return RORBK_OK;
    int32_t *d = nullptr;
    CHK(dalloc(&d, (size_t)(3 * count)));
    hipError_t e1 = launch_sample(seed, j0, count, h->d_W, h->L.k, d, h->stream);
    hipError_t e2 = hipMemcpyAsync(tau_host, d, 4 * 3 * count, hipMemcpyDeviceToHost, h->stream);
    hipError_t e3 = hipStreamSynchronize(h->stream);
    dfree(d);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return fail(RORBK_ERR_HIP, "sampling failed");
    return RORBK_OK;
}

int ror_bk_topk(rorbk_handle h, const void *r, int32_t vec_f32, int32_t *idx) {
    if (!h || !r || !idx) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    const int vec = vec_f32 ? VEC_F32 : VEC_F64;
    HIPCHK(hipMemsetAsync(h->d_ctrl, 0, sizeof(Ctrl), h->stream));
    SelectArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.vec = vec;
    sa.b = r;
    sa.axp = nullptr;
    sa.r = h->d_r;
    sa.it = 0;
    sa.I_out = idx;
    sa.rI_out = h->d_rI;
    sa.stop_test = 0;
    HIPCHK(launch_select(h, sa, h->stream));
    HIPCHK(hipMemcpyAsync(h->h_ctrl, h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (h->h_ctrl->status) return fail(h->h_ctrl->status, "non-finite entry in r");
    return RORBK_OK;
}

int ror_bk_residual(rorbk_handle h, const void *b, const void *x, void *r, double *block_norm2,
                    int32_t vec_f32, int32_t use_f64_master, double *rrn_host) {
    if (!h || !b || !x || !r) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    const Layout &L = h->L;
    const int vec = vec_f32 ? VEC_F32 : VEC_F64;
    const void *A = h->A;
    int dt = L.dtype, al = h->aligned;
    if (use_f64_master || (vec == VEC_F64 && L.dtype != RORBK_F64)) {
        if (!h->A64) return fail(RORBK_ERR_INVALID_ARG, "no FP64 master copy");
        A = h->A64;
        dt = RORBK_F64;
        al = h->aligned64;
    }
    if (vec == VEC_F32 && dt == RORBK_F64)
        return fail(RORBK_ERR_INVALID_ARG, "float vectors need F32 or BF16 storage");
    HIPCHK(hipMemsetAsync(h->d_ctrl, 0, sizeof(Ctrl), h->stream));
    HIPCHK(launch_norm2(b, vec, L.m, h->d_red, h->d_red, h->stream));
    HIPCHK(launch_init_ctrl(h->d_ctrl, 0.0, h->d_red, h->stream));
    HIPCHK(residual(h, A, dt, al, vec, x, h->d_axp));
    SelectArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.vec = vec;
    sa.b = b;
    sa.axp = h->d_axp;
    sa.nseg = L.nseg;
    sa.r = r;
    sa.skip_topk = 1;
    HIPCHK(launch_select(h, sa, h->stream));
    if (block_norm2)
        HIPCHK(hipMemcpyAsync(block_norm2, h->d_bn, 8 * L.k, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->h_ctrl, h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const Ctrl &c = *h->h_ctrl;
    if (rrn_host) *rrn_host = c.bnorm2 > 0 ? std::sqrt(c.rnorm2 / c.bnorm2) : 0.0;
    if (c.status) return fail(c.status, "non-finite residual");
    return RORBK_OK;
}

int ror_bk_fabgmres(rorbk_handle h, const double *b, double *x, uint64_t seed, double tol,
                    int64_t max_outer, int64_t inner_iters, double eta, rorbk_info *info) {
    g_msg[0] = 0;
    if (!h || !b || !x) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    if (max_outer < 1 || inner_iters < 1)
        return fail(RORBK_ERR_INVALID_ARG, "max_outer and inner_iters must be >= 1");
    if (!(tol >= 0.0) || !std::isfinite(tol) || !(eta >= 0.0) || !std::isfinite(eta))
        return fail(RORBK_ERR_INVALID_ARG, "tol and eta must be finite and >= 0");
    const Layout &L = h->L;
    if (L.dtype != RORBK_F64)
        return fail(RORBK_ERR_UNSUPPORTED, "flexible AB-GMRES runs on FP64 storage");
    hipStream_t s = h->stream;
    const int64_t m = L.m, n = L.n, M1 = max_outer + 1;
    h->rec_valid = 0;
    h->rec_I_valid = 0;
    h->rec_iters = 0;
    h->profile = 0;
    // workspaces of this call
    double *V = nullptr, *Z = nullptr, *small = nullptr;
    int rc = dalloc(&V, (size_t)(m * M1));
    if (!rc) rc = dalloc(&Z, (size_t)(n * max_outer));
    // hcol (M1), R (M1 * max_outer), cs, sn (max_outer), g (M1), est (2), beta (1),
    // the Gram-Schmidt partial sums (256)
    const size_t nsmall = (size_t)(M1 + M1 * max_outer + 2 * max_outer + M1 + 3 + 256);
    if (!rc) rc = dalloc(&small, nsmall);
    if (!rc) rc = ensure_solve_buffers(h, inner_iters, false, 0, VEC_F64);
    auto cleanup = [&]() {
        dfree(V);
        dfree(Z);
        dfree(small);
    };
    if (rc) {
        cleanup();
        return rc;
    }
    double *hcol = small, *R = hcol + M1, *cs = R + M1 * max_outer, *sn = cs + max_outer;
    double *g = sn + max_outer, *est = g + M1, *beta_d = est + 2, *gs_part = beta_d + 1;
#define GCHK(expr)                                                                   \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            cleanup();                                                               \
            return fail(RORBK_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));      \
        }                                                                            \
    } while (0)
    GCHK(launch_fill_zero(small, (int64_t)(sizeof(double) * nsmall), s));
    GCHK(launch_fill_zero(Z, (int64_t)(sizeof(double) * n * max_outer), s));
    // ||b|| and r0 = b - A x0, v_1 = r0 / beta
    GCHK(launch_norm2(b, VEC_F64, m, h->d_red, h->d_red + 1, s));
    GCHK(hipMemsetAsync(h->d_ctrl, 0, sizeof(Ctrl), s));
    GCHK(residual(h, h->A, RORBK_F64, h->aligned, VEC_F64, x, h->d_axp));
    GCHK(launch_gmres_start(b, h->d_axp, L.nseg, m, V, g, beta_d, s));
    double hb[2] = {0.0, 0.0};
    GCHK(hipMemcpyAsync(&hb[0], h->d_red + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    GCHK(hipMemcpyAsync(&hb[1], beta_d, sizeof(double), hipMemcpyDeviceToHost, s));
    GCHK(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(hb[0]);
    int64_t kend = 0, inner_total = 0;
    bool conv = false;
    if (hb[1] > 0.0) {
        for (int64_t k = 0; k < max_outer; ++k) {
            double *vk = V + k * m, *zk = Z + k * n;
            // z_k: ROR-BK on A z = v_k from zero, sampler counter from k * inner_iters
            int prc = prepare_tau(h, seed, k * inner_iters, inner_iters, false);
            if (prc) { cleanup(); return prc; }
            GCHK(launch_norm2(vk, VEC_F64, m, h->d_red, h->d_red + 2, s));
            GCHK(launch_init_ctrl(h->d_ctrl, eta, h->d_red + 2, s));
            RunOpts o;
            memset(&o, 0, sizeof(o));
            o.vec = VEC_F64;
            o.A = h->A;
            o.dt = RORBK_F64;
            o.aligned = h->aligned;
            o.b = vk;
            o.x = zk;
            int64_t ran = 0;
            bool stopped = false;
            int irc = run_iterations(h, o, 0, inner_iters, &ran, &stopped);
            if (irc) { cleanup(); return irc; }
            inner_total += ran;
            // w = A z_k, Gram-Schmidt, Givens
            GCHK(hipMemsetAsync(h->d_ctrl, 0, sizeof(Ctrl), s));
            GCHK(residual(h, h->A, RORBK_F64, h->aligned, VEC_F64, zk, h->d_axp));
            GCHK(launch_gmres_step(V, m, (int)k, h->d_axp, L.nseg, hcol, (int)M1, R, cs, sn, g,
                                   est, gs_part, s));
            double he[2];
            GCHK(hipMemcpyAsync(he, est, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            GCHK(hipStreamSynchronize(s));
            kend = k + 1;
            if (he[0] < tol * bnorm) {
                conv = true;
                break;
            }
            if (he[1] == 0.0) break;
        }
        GCHK(launch_gmres_update(Z, n, R, g, (int)kend, (int)M1, x, s));
    } else {
        conv = true;
    }
    // the true relative residual of the result
    GCHK(hipMemsetAsync(h->d_ctrl, 0, sizeof(Ctrl), s));
    GCHK(launch_init_ctrl(h->d_ctrl, 0.0, h->d_red + 1, s));
    GCHK(residual(h, h->A, RORBK_F64, h->aligned, VEC_F64, x, h->d_axp));
    SelectArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.vec = VEC_F64;
    sa.b = b;
    sa.axp = h->d_axp;
    sa.nseg = L.nseg;
    sa.r = h->d_r64;
    sa.skip_topk = 1;
    GCHK(launch_select(h, sa, s));
    GCHK(hipMemcpyAsync(h->h_ctrl, h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    GCHK(hipStreamSynchronize(s));
#undef GCHK
    cleanup();
    if (info) {
        memset(info, 0, sizeof(*info));
        info->iters = inner_total;
        info->n_refine = (int32_t)kend;
        info->converged = conv ? 1 : 0;
        const Ctrl &c = *h->h_ctrl;
        info->rrn = c.bnorm2 > 0 ? std::sqrt(c.rnorm2 / c.bnorm2) : 0.0;
        info->rrn_test = info->rrn;
        info->t_setup_s = h->t_setup_s;
    }
    return RORBK_OK;
}

int ror_bk_initial_solution(rorbk_handle h, const void *b, void *x0, int32_t vec_f32,
                            double *coef_host) {
    if (!h || !b || !x0) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    g_msg[0] = 0;
    const Layout &L = h->L;
    const int vec = vec_f32 ? VEC_F32 : VEC_F64;
    const void *A = h->A;
    int dt = L.dtype, al = h->aligned;
    if (vec == VEC_F64 && L.dtype != RORBK_F64) {
        if (!h->A64) return fail(RORBK_ERR_INVALID_ARG, "FP64 vectors need the FP64 master copy");
        A = h->A64;
        dt = RORBK_F64;
        al = h->aligned64;
    }
    if (vec == VEC_F32 && dt == RORBK_F64)
        return fail(RORBK_ERR_INVALID_ARG, "float vectors need F32 or BF16 storage");
    const void *yv = h->d_ysum;
    if (vec == VEC_F32) {
        if (!h->d_ysum32) CHK(dalloc(&h->d_ysum32, (size_t)L.n));
        HIPCHK(launch_cast_f64_to_f32(h->d_ysum, h->d_ysum32, L.n, h->stream));
        yv = h->d_ysum32;
    }
    HIPCHK(hipMemsetAsync(h->d_ctrl, 0, sizeof(Ctrl), h->stream));   // the product pass runs
    HIPCHK(residual(h, A, dt, al, vec, yv, h->d_axp));
    HIPCHK(launch_alg2(b, vec, h->d_axp, L.nseg, L.m, h->d_ysum, h->d_alg2, x0, L.n, h->stream));
    if (coef_host) {
        HIPCHK(hipMemcpyAsync(coef_host, h->d_alg2 + 2, sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return RORBK_OK;
}

int ror_bk_set_replay(rorbk_handle h, const int32_t *tau_host, const int32_t *I_host,
                      int64_t iters) {
    if (!h || !tau_host || !I_host || iters < 1)
        return fail(RORBK_ERR_INVALID_ARG, "bad replay arguments");
    const Layout &L = h->L;
    for (int64_t i = 0; i < 3 * iters; ++i)
        if (tau_host[i] < 0 || tau_host[i] >= L.k)
            return fail(RORBK_ERR_INVALID_ARG, "replayed tau[%lld] = %d outside [0, %lld)",
                        (long long)i, tau_host[i], (long long)L.k);
    for (int64_t it = 0; it < iters; ++it)
        for (int64_t p = 0; p < L.K; ++p) {
            const int32_t v = I_host[it * L.K + p];
            if (v < 0 || v >= L.m || (p > 0 && v <= I_host[it * L.K + p - 1]))
                return fail(RORBK_ERR_INVALID_ARG,
                            "replayed greedy set %lld is not ascending within [0, m)", (long long)it);
        }
    dfree(h->d_rep_tau);
    dfree(h->d_rep_I);
    h->rep_iters = 0;
    CHK(dalloc(&h->d_rep_tau, (size_t)(3 * iters)));
    CHK(dalloc(&h->d_rep_I, (size_t)(iters * L.K)));
    HIPCHK(hipMemcpyAsync(h->d_rep_tau, tau_host, 4 * 3 * iters, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_rep_I, I_host, 4 * iters * L.K, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->rep_iters = iters;
    return RORBK_OK;
}

int ror_bk_get_profile(rorbk_handle h, double *out4_host) {
    if (!h || !out4_host) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    out4_host[0] = h->prof_in_n ? h->prof_in_ms / (double)h->prof_in_n : 0.0;
    out4_host[1] = (double)h->prof_in_n;
    out4_host[2] = h->prof_out_n ? h->prof_out_ms / (double)h->prof_out_n : 0.0;
    out4_host[3] = (double)h->prof_out_n;
    return RORBK_OK;
}

int ror_bk_set_refine(rorbk_handle h, int64_t inner_iters, double eta) {
    if (!h || inner_iters < 1 || !(eta >= 0.0) || !std::isfinite(eta))
        return fail(RORBK_ERR_INVALID_ARG, "bad refinement arguments");
    h->refine_inner = inner_iters;
    h->refine_eta = eta;
    return RORBK_OK;
}

int ror_bk_get_record(rorbk_handle h, int32_t *tau_host, int32_t *I_host, double *rrn_host,
                      int64_t *iters_host) {
    if (!h) return fail(RORBK_ERR_INVALID_ARG, "NULL handle");
    const int64_t it = h->rec_iters;
    if (iters_host) *iters_host = it;
    if (it == 0) return RORBK_OK;
    if (tau_host) HIPCHK(hipMemcpyAsync(tau_host, h->d_tau, 4 * 3 * it, hipMemcpyDeviceToHost, h->stream));
    if (I_host) {
        if (!h->d_recI || !h->rec_I_valid)
            return fail(RORBK_ERR_NOT_RECORDED, "the last solve did not record its greedy sets");
        HIPCHK(hipMemcpyAsync(I_host, h->d_recI, 4 * it * h->L.K, hipMemcpyDeviceToHost, h->stream));
    }
    if (rrn_host) HIPCHK(hipMemcpyAsync(rrn_host, h->d_recR, 8 * it, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RORBK_OK;
}

int ror_bk_solve(rorbk_handle h, const void *b, void *x, uint64_t seed, double tol,
                 int64_t max_iters, int64_t start_iter, uint32_t flags, int64_t checkpoint_every,
                 rorbk_info *info) {
    g_msg[0] = 0;
    if (!h || !b || !x) return fail(RORBK_ERR_INVALID_ARG, "NULL handle or vector");
    if (max_iters < 0 || start_iter < 0)
        return fail(RORBK_ERR_INVALID_ARG, "max_iters and start_iter must be >= 0");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(RORBK_ERR_INVALID_ARG, "tol must be finite, >= 0");
    if (flags & ~(RORBK_REFINE | RORBK_RECORD | RORBK_REPLAY | RORBK_CHECKPOINT | RORBK_PROFILE))
        return fail(RORBK_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const bool refine = flags & RORBK_REFINE, record = flags & RORBK_RECORD;
    const bool replay = flags & RORBK_REPLAY, ckpt = flags & RORBK_CHECKPOINT;
    if (refine && (record || replay || ckpt))
        return fail(RORBK_ERR_INVALID_ARG, "REFINE cannot be combined with RECORD, REPLAY or CHECKPOINT");
    if (ckpt && checkpoint_every < 1)
        return fail(RORBK_ERR_INVALID_ARG, "CHECKPOINT needs checkpoint_every >= 1");
    if (replay && h->rep_iters < max_iters)
        return fail(RORBK_ERR_INVALID_ARG, "replay table holds %lld iterations, %lld requested",
                    (long long)h->rep_iters, (long long)max_iters);
    if (refine && !h->A64)
        return fail(RORBK_ERR_INVALID_ARG, "REFINE needs the FP64 master copy (values_f64)");
    const Layout &L = h->L;
    hipStream_t s = h->stream;
    rorbk_info inf;
    memset(&inf, 0, sizeof(inf));
    inf.rrn = NAN;
    inf.rrn_test = NAN;
    inf.t_setup_s = h->t_setup_s;
    h->rec_valid = 0;
    h->rec_I_valid = 0;
    h->rec_iters = 0;
    h->profile = (flags & RORBK_PROFILE) ? 1 : 0;
    h->prof_in_ms = h->prof_out_ms = 0.0;
    h->prof_in_n = h->prof_out_n = 0;
    if (max_iters == 0) {
        if (info) *info = inf;
        return RORBK_OK;
    }
    const int vec_work = (L.dtype == RORBK_F64) ? VEC_F64 : VEC_F32;
    const int vec = refine ? VEC_F64 : vec_work;
    const int64_t slots = ckpt ? (max_iters + checkpoint_every - 1) / checkpoint_every : 0;
    CHK(ensure_solve_buffers(h, max_iters, record || ckpt, slots, vec));
    CHK(prepare_tau(h, seed, start_iter, max_iters, replay));
    // ||b|| and the stop threshold
    HIPCHK(launch_norm2(b, vec, L.m, h->d_red, h->d_red + 1, s));
    HIPCHK(launch_init_ctrl(h->d_ctrl, tol, h->d_red + 1, s));
    hipEvent_t t0, t1;
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    HIPCHK(hipEventRecord(t0, s));
    int rc = RORBK_OK;
    if (!refine) {
        RunOpts o;
        memset(&o, 0, sizeof(o));
        o.vec = vec;
        o.A = h->A;
        o.dt = L.dtype;
        o.aligned = h->aligned;
        o.b = b;
        o.x = x;
        o.record_I = record || ckpt;
        o.replay_I = replay ? h->d_rep_I : nullptr;
        o.ckpt_every = ckpt ? checkpoint_every : 0;
        o.ckpt = h->d_ckpt;
        int64_t ran = 0;
        bool stopped = false;
        rc = run_iterations(h, o, 0, max_iters, &ran, &stopped);
        if (rc == RORBK_OK) {
            inf.iters = ran;
            inf.converged = stopped ? 1 : 0;
            const Ctrl c = *h->h_ctrl;
            inf.rrn_test = c.bnorm2 > 0 ? std::sqrt(c.rnorm2 / c.bnorm2) : 0.0;
            inf.rrn = inf.rrn_test;
            h->rec_iters = ran;
            if (record || ckpt) {
                h->rec_valid = ckpt ? 2 : 1;
                h->rec_I_valid = 1;
                h->rec_converged = inf.converged;
                h->ckpt_every = ckpt ? checkpoint_every : 0;
                h->rec_b = b;
                h->rec_seed = seed;
                h->rec_vec = vec;
                h->rec_thr = c.thr;
            }
            if (!stopped) {
                // the greedy update after the last stop test changed x: one
                // more residual pass measures the iterate returned
                HIPCHK(residual(h, h->A, L.dtype, h->aligned, vec, x, h->d_axp));
                SelectArgs sa;
                memset(&sa, 0, sizeof(sa));
                sa.vec = vec;
                sa.b = b;
                sa.axp = h->d_axp;
                sa.nseg = L.nseg;
                sa.r = h->d_r;
                sa.skip_topk = 1;
                HIPCHK(launch_select(h, sa, s));
                HIPCHK(hipMemcpyAsync(h->h_ctrl, h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                const Ctrl &cf = *h->h_ctrl;
                if (cf.status) return fail(cf.status, "non-finite residual of the returned x");
                inf.rrn = cf.bnorm2 > 0 ? std::sqrt(cf.rnorm2 / cf.bnorm2) : 0.0;
            }
        }
    } else {
        // FP64 outer residual with the master copy; inner ROR-BK on the working
        // storage against r_out from d = 0 (restart-equivalent to continuing
        // on A x = b), then x += d.  The RNG counter runs on across steps.
        const int vin = vec_work;
        double bnorm2 = 0.0;
        HIPCHK(hipMemcpyAsync(&h->h_ctrl[0], h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bnorm2 = h->h_ctrl[0].bnorm2;
        const double thr = tol * std::sqrt(bnorm2);
        if (!h->d_rhs32) {
            char *p1 = nullptr, *p2 = nullptr;
            CHK(dalloc(&p1, (size_t)(8 * L.m)));
            h->d_rhs32 = p1;
            CHK(dalloc(&p2, (size_t)(8 * L.n)));
            h->d_d32 = p2;
        }
        int64_t total = 0;
        int nref = 0;
        double rrn = NAN;
        bool conv = false;
        for (;;) {
            HIPCHK(launch_init_ctrl(h->d_ctrl, tol, h->d_red + 1, s));
            if (h->profile) HIPCHK(hipEventRecord(h->evr[0][0], s));
            HIPCHK(residual(h, h->A64, RORBK_F64, h->aligned64, VEC_F64, x, h->d_axp));
            if (h->profile) HIPCHK(hipEventRecord(h->evr[0][1], s));
            SelectArgs sa;
            memset(&sa, 0, sizeof(sa));
            sa.vec = VEC_F64;
            sa.b = b;
            sa.axp = h->d_axp;
            sa.nseg = L.nseg;
            sa.r = h->d_r64;
            sa.skip_topk = 1;
            HIPCHK(launch_select(h, sa, s));
            HIPCHK(hipMemcpyAsync(&h->h_ctrl[0], h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (h->profile) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, h->evr[0][0], h->evr[0][1]));
                h->prof_out_ms += ms;
                h->prof_out_n += 1;
            }
            const Ctrl c = h->h_ctrl[0];
            if (c.status) {
                rc = fail(c.status, "non-finite FP64 residual");
                break;
            }
            const double rn = std::sqrt(c.rnorm2);
            rrn = bnorm2 > 0 ? rn / std::sqrt(bnorm2) : 0.0;
            if (rn < thr) { conv = true; break; }
            if (total >= max_iters) break;
            const int64_t cnt = std::min(h->refine_inner, max_iters - total);
            // inner right-hand side and zero correction
            if (vin == VEC_F32) {
                HIPCHK(launch_cast_f64_to_f32(h->d_r64, (float *)h->d_rhs32, L.m, s));
            } else {
                HIPCHK(hipMemcpyAsync(h->d_rhs32, h->d_r64, 8 * L.m, hipMemcpyDeviceToDevice, s));
            }
            HIPCHK(launch_fill_zero(h->d_d32, (int64_t)(L.n * vec_size(vin)), s));
            // ||r_out||^2 for the inner threshold
            HIPCHK(hipMemcpyAsync(h->d_red + 2, &h->h_ctrl[0].rnorm2, 8, hipMemcpyHostToDevice, s));
            HIPCHK(launch_set_refine_ctrl(h->d_ctrl, tol, h->refine_eta, h->d_red + 2, bnorm2, s));
            RunOpts o;
            memset(&o, 0, sizeof(o));
            o.vec = vin;
            o.A = h->A;
            o.dt = L.dtype;
            o.aligned = h->aligned;
            o.b = h->d_rhs32;
            o.x = h->d_d32;
            int64_t ran = 0;
            bool stopped = false;
            rc = run_iterations(h, o, total, total + cnt, &ran, &stopped);
            if (rc) break;
            if (vin == VEC_F32) {
                HIPCHK(launch_axpy_f32_to_f64((const float *)h->d_d32, (double *)x, L.n, s));
            } else {
                HIPCHK(launch_axpy_f64((const double *)h->d_d32, (double *)x, L.n, s));
            }
            total += ran;
            ++nref;
        }
        inf.iters = total;
        inf.converged = conv ? 1 : 0;
        inf.rrn = rrn;
        inf.rrn_test = rrn;
        inf.n_refine = nref;
        h->rec_iters = total;
    }
    HIPCHK(hipEventRecord(t1, s));
    HIPCHK(hipEventSynchronize(t1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    inf.t_solve_s = ms * 1e-3;
    if (info) *info = inf;
    return rc;
}

// Adjoint of the recorded iteration (see the header).  The steps of iteration
// `it`, newest first: the greedy one (absent in a converged last iteration)
// then the three sampled ones.  Each step consumes the partial products
// A_S g of its rows, produced by the previous kernel.
namespace {

int backward_range(rorbk_handle_s *h, int64_t a, int64_t bnd, bool last_conv_in_range,
                   void *g, void *gb, int vec, int *ping_io, bool first) {
    const Layout &L = h->L;
    hipStream_t s = h->stream;
    int ping = *ping_io;
    // steps in reverse order as a list of RowSel
    struct St { RowSel r; int greedy; int64_t it; };
    std::vector<St> steps;
    for (int64_t it = bnd - 1; it >= a; --it) {
        const bool has_greedy = !(last_conv_in_range && it == bnd - 1);
        if (has_greedy) {
            St st;
            st.r.kind = 1;
            st.r.count = (int32_t)L.K;
            st.r.tau_index = 0;
            st.r.idx = h->d_recI + it * L.K;
            st.greedy = 1;
            st.it = it;
            steps.push_back(st);
        }
        for (int l = 2; l >= 0; --l) {
            St st;
            st.r.kind = 0;
            st.r.count = 0;
            st.r.tau_index = 3 * it + l;
            st.r.idx = nullptr;
            st.greedy = 0;
            st.it = it;
            steps.push_back(st);
        }
    }
    if (steps.empty()) return RORBK_OK;
    StepArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.A = h->A;
    sa.dt = L.dtype;
    sa.aligned = h->aligned;
    sa.vec = vec;
    sa.b = nullptr;
    sa.x = g;
    sa.gb = gb;
    (void)first;
    // partial products of the first step
    sa.cur.kind = -1;
    sa.ymode = 2;
    sa.nxt = steps[0].r;
    sa.Pout = h->d_P[ping ^ 1];
    HIPCHK(step(h, sa));
    ping ^= 1;
    for (size_t i = 0; i < steps.size(); ++i) {
        const St &st = steps[i];
        sa.cur = st.r;
        if (h->col) {
            // column form: y = -A_S (A_S^T A_S + lambda I)^{-1} g, gb[S] -= y
            HIPCHK(launch_col_adjoint(h, st.r, vec, g, gb, h->d_bigr, s));
            sa.ymode = 3;
            sa.ygiven = h->d_bigr;
        } else if (st.greedy) {
            HIPCHK(gram(h, h->A, L.dtype, h->aligned, st.r.idx, (int)L.K, h->d_G));
            HIPCHK(launch_chol_solve(h, h->d_G, (int)L.K, nullptr, h->d_P[ping], h->d_y, s));
            sa.ymode = 1;
            sa.ygiven = h->d_y;
        } else {
            sa.ymode = 0;
            sa.Pin = h->d_P[ping];
        }
        if (i + 1 < steps.size()) {
            sa.nxt = steps[i + 1].r;
            sa.Pout = h->d_P[ping ^ 1];
        } else {
            sa.nxt.kind = -1;
            sa.Pout = nullptr;
        }
        HIPCHK(step(h, sa));
        if (i + 1 < steps.size()) ping ^= 1;
    }
    *ping_io = ping;
    return RORBK_OK;
}

}  // namespace

int ror_bk_backward(rorbk_handle h, const void *grad_x, void *grad_b, void *grad_x0) {
    g_msg[0] = 0;
    if (!h || !grad_x || !grad_b || !grad_x0) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    if (!h->rec_valid) return fail(RORBK_ERR_NOT_RECORDED, "no RECORD or CHECKPOINT solve to differentiate");

    const Layout &L = h->L;
    hipStream_t s = h->stream;
    const int vec = h->rec_vec;
    const size_t vs = vec_size(vec);
    const int64_t iters = h->rec_iters;
    const bool conv = h->rec_converged != 0;
    HIPCHK(hipMemcpyAsync(grad_x0, grad_x, L.n * vs, hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_fill_zero(grad_b, (int64_t)(L.m * vs), s));
    HIPCHK(hipMemsetAsync(h->d_ctrl, 0, sizeof(Ctrl), s));
    int ping = 0;
    if (h->rec_valid == 1) {
        CHK(backward_range(h, 0, iters, conv, grad_x0, grad_b, vec, &ping, true));
    } else {
        const int64_t c = h->ckpt_every;
        const int64_t nseg = (iters + c - 1) / c;
        char *xw = nullptr;
        CHK(dalloc(&xw, (size_t)(L.n * vs)));
        double *bn2 = h->d_red + 3;
        int rc = RORBK_OK;
        for (int64_t sg = nseg - 1; sg >= 0 && rc == RORBK_OK; --sg) {
            const int64_t a = sg * c, e = std::min(iters, a + c);
            // recompute the segment's greedy sets from its checkpoint
            hipError_t he = hipMemcpyAsync(xw, (char *)h->d_ckpt + (size_t)sg * L.n * vs, L.n * vs,
                                           hipMemcpyDeviceToDevice, s);
            if (he == hipSuccess) he = launch_norm2(h->rec_b, vec, L.m, h->d_red, bn2, s);
            if (he == hipSuccess) he = launch_init_ctrl(h->d_ctrl, 0.0, bn2, s);
            if (he != hipSuccess) { rc = fail(RORBK_ERR_HIP, "checkpoint restore failed"); break; }
            // same threshold as the recorded solve
            Ctrl hc;
            memset(&hc, 0, sizeof(hc));
            RunOpts o;
            memset(&o, 0, sizeof(o));
            o.vec = vec;
            o.A = h->A;
            o.dt = L.dtype;
            o.aligned = h->aligned;
            o.b = h->rec_b;
            o.x = xw;
            o.record_I = true;
            rc = launch_set_thr(h->d_ctrl, h->rec_thr, s) == hipSuccess ? RORBK_OK
                     : fail(RORBK_ERR_HIP, "threshold restore failed");
            if (rc) break;
            if (h->chain && sg > 0) {
                // the checkpoint holds the chain state of iteration a: restore
                // the greedy rows, y and z, form the cross-Grams of a's blocks
                // as the forward did, and take a's sampled steps together
                // with the greedy update of a - 1, as the forward did
                const double *st = h->d_ckst + sg * CKST_DOUBLES;
                he = hipMemcpyAsync(h->d_I, st, L.K * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
                if (he == hipSuccess)
                    he = hipMemcpyAsync(h->d_y, st + 32, L.K * sizeof(double),
                                        hipMemcpyDeviceToDevice, s);
                if (he == hipSuccess)
                    he = hipMemcpyAsync(h->d_z3, st + 96, 3 * RORBK_FWD_MAX_BLOCK * sizeof(double),
                                        hipMemcpyDeviceToDevice, s);
                double *xga = h->d_XG + (a & 1) * 3 * L.bmax * L.bmax;
                if (he == hipSuccess)
                    he = launch_xgram(h, h->A, L.dtype, h->aligned, 3 * a, xga, 8, s);
                if (he == hipSuccess) {
                    FwdArgs fa;
                    memset(&fa, 0, sizeof(fa));
                    fa.A = h->A;
                    fa.dt = L.dtype;
                    fa.aligned = h->aligned;
                    fa.vec = vec;
                    fa.b = h->rec_b;
                    fa.x = xw;
                    fa.I = h->d_I;
                    fa.y = h->d_y;
                    fa.tau_index = 3 * a;
                    fa.xg = xga;
                    he = launch_fwd_samp3(h, fa, s);
                }
                if (he != hipSuccess) { rc = fail(RORBK_ERR_HIP, "chain state restore failed"); break; }
                o.resume_chain = true;
            }
            int64_t ran = 0;
            bool stopped = false;
            rc = run_iterations(h, o, a, e, &ran, &stopped);
            if (rc) break;
            HIPCHK(hipMemsetAsync(h->d_ctrl, 0, sizeof(Ctrl), s));
            rc = backward_range(h, a, e, conv && e == iters, grad_x0, grad_b, vec, &ping, sg == nseg - 1);
        }
        (void)hipStreamSynchronize(s);
        dfree(xw);
        if (rc) return rc;
    }
    HIPCHK(hipMemcpyAsync(h->h_ctrl, h->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h->h_ctrl->status) return fail(h->h_ctrl->status, "backward failed (block Gram not SPD)");
    return RORBK_OK;
}

}  // extern "C"

// ============================================ residual pass without allocation
// ror_bk_residual_noalloc: the residual pass of ror_bk_residual for callers
// that cannot allocate device memory.  Its workspace (control block, the
// selection counter, norms, the residual's partial products) lives in the
// file-scope array below, one copy per GPU, held until the process ends.  Host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device (looked up on the first call on that device); the
// array's own name is a host-side stand-in and is never passed to a kernel.
static __device__ __align__(256) unsigned char scratch[RORBK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t NOALLOC_BYTES = RORBK_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEV = 64;

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEV] = {};
int g_noalloc_ncu[NOALLOC_MAX_DEV] = {};

// The current device's copy of the scratch array and its compute-unit count.
int noalloc_scratch(void **ptr, int *ncu) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEV)
        return fail(RORBK_ERR_UNSUPPORTED, "device %d beyond the %d devices supported", dev,
                    NOALLOC_MAX_DEV);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(RORBK_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        g_noalloc_ncu[dev] = n;
        g_noalloc_ptr[dev] = p;
    }
    *ptr = g_noalloc_ptr[dev];
    *ncu = g_noalloc_ncu[dev];
    return RORBK_OK;
}

__global__ void k_rrn_out(const Ctrl *__restrict__ c, double *__restrict__ rrn) {
    const double bn2 = c->bnorm2;
    *rrn = bn2 > 0.0 ? sqrt(c->rnorm2 / bn2) : 0.0;
}

size_t round256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

extern "C" int ror_bk_residual_noalloc(const rorbk_matrix *A, int64_t block_rows, const void *b,
                                       const void *x, void *r, double *block_norm2, double *rrn,
                                       int32_t vec_f32, void *stream) {
    g_msg[0] = 0;
    // ---- host-side checks (nothing touches the device before they pass)
    if (!A || !b || !x || !r) return fail(RORBK_ERR_INVALID_ARG, "NULL argument");
    if (A->format != RORBK_DENSE && A->format != RORBK_CSR)
        return fail(RORBK_ERR_INVALID_ARG, "unknown format %d", A->format);
    if (A->dtype != RORBK_F64 && A->dtype != RORBK_F32 && A->dtype != RORBK_BF16)
        return fail(RORBK_ERR_INVALID_ARG, "unknown dtype %d", A->dtype);
    if (A->m < 1 || A->n < 1) return fail(RORBK_ERR_INVALID_ARG, "empty matrix");
    if (A->m > INT32_MAX || A->n > INT32_MAX)
        return fail(RORBK_ERR_UNSUPPORTED, "dimensions above 2^31 are not supported");
    const bool dense = A->format == RORBK_DENSE;
    if (dense && A->ld < A->n)
        return fail(RORBK_ERR_INVALID_ARG, "ld %lld < n %lld", (long long)A->ld, (long long)A->n);
    if (!dense) {
        if (!A->rowptr || A->nnz < 0)
            return fail(RORBK_ERR_INVALID_ARG, "CSR needs rowptr and nnz >= 0");
        if (A->dtype == RORBK_BF16) return fail(RORBK_ERR_UNSUPPORTED, "BF16 storage is dense only");
        if (A->nnz > 0 && (!A->colidx || !A->values))
            return fail(RORBK_ERR_INVALID_ARG, "CSR with nnz > 0 needs colidx and values");
    }
    if (block_rows < 1 || block_rows > A->m)
        return fail(RORBK_ERR_INVALID_ARG, "block_rows %lld outside [1, m=%lld]",
                    (long long)block_rows, (long long)A->m);
    const int vec = vec_f32 ? VEC_F32 : VEC_F64;
    const void *Am = A->values;
    int dt = A->dtype;
    if (vec == VEC_F64 && dt != RORBK_F64) {
        if (!A->values_f64) return fail(RORBK_ERR_INVALID_ARG, "double vectors need values_f64");
        Am = A->values_f64;
        dt = RORBK_F64;
    }
    if (vec == VEC_F32 && dt == RORBK_F64)
        return fail(RORBK_ERR_INVALID_ARG, "float vectors need F32 or BF16 storage");
    if (!Am && !(!dense && A->nnz == 0)) return fail(RORBK_ERR_INVALID_ARG, "matrix values are NULL");

    rorbk_handle_s hh;
    memset(&hh, 0, sizeof(hh));
    Layout &L = hh.L;
    L.m = A->m;
    L.n = A->n;
    L.ld = dense ? A->ld : A->n;
    L.nnz = A->nnz;
    L.format = A->format;
    L.dtype = A->dtype;
    L.k = A->m / block_rows;
    L.q = A->m / L.k;
    L.rem = A->m - L.k * L.q;
    L.K = L.q;
    L.bmax = L.q + (L.rem > 0 ? 1 : 0);
    if (L.bmax > RORBK_MAX_BIG_BLOCK_ROWS)
        return fail(RORBK_ERR_UNSUPPORTED, "blocks of %lld rows exceed the supported %d",
                    (long long)L.bmax, RORBK_MAX_BIG_BLOCK_ROWS);
    L.nseg = dense ? (int32_t)((L.n + 2047) / 2048) : 1;
    L.bpc = sel_blocks_per_chunk(L.k, L.bmax, L.nseg);
    L.nch_s = (int32_t)((L.k + L.bpc - 1) / L.bpc);
    // scratch layout: control block, counter, norm scratch | chunk norms |
    // block norms (unless the caller takes them) | partial products
    const size_t off_cn = 1024;
    const size_t off_bn = off_cn + round256(8 * (size_t)L.nch_s);
    const size_t off_axp = off_bn + (block_norm2 ? 0 : round256(8 * (size_t)L.k));
    const size_t need = off_axp + round256(8 * (size_t)L.nseg * (size_t)L.m);
    if (need > NOALLOC_BYTES)
        return fail(RORBK_ERR_UNSUPPORTED,
                    "needs %zu bytes of scratch (8 x %d segments x %lld rows of partial products "
                    "plus norms), above the %zu bytes of the static array",
                    need, L.nseg, (long long)L.m, NOALLOC_BYTES);

    // ---- device work, enqueued on the caller's stream; no allocation
    void *base = nullptr;
    CHK(noalloc_scratch(&base, &hh.ncu));
    char *sb = (char *)base;
    hh.stream = (hipStream_t)stream;
    hh.A = A->values;
    hh.rowptr = A->rowptr;
    hh.colidx = A->colidx;
    hh.d_ctrl = (Ctrl *)sb;
    hh.d_selcnt = (uint32_t *)(sb + 256);
    hh.d_red = (double *)(sb + 512);
    hh.d_cn = (double *)(sb + off_cn);
    hh.d_bn = block_norm2 ? block_norm2 : (double *)(sb + off_bn);
    hh.d_axp = (double *)(sb + off_axp);
    const int al = (dense && aligned16(Am, L.ld, dtype_size(dt))) ? 1 : 0;
    hipStream_t s = hh.stream;
    // the counter must start at zero (a fill kernel, not a memset node)
    HIPCHK(launch_fill_zero(hh.d_selcnt, 4, s));
    HIPCHK(launch_norm2(b, vec, L.m, hh.d_red, hh.d_red, s));
    HIPCHK(launch_init_ctrl(hh.d_ctrl, 0.0, hh.d_red, s));
    HIPCHK(residual(&hh, Am, dt, al, vec, x, hh.d_axp));
    SelectArgs sa;
    memset(&sa, 0, sizeof(sa));
    sa.vec = vec;
    sa.b = b;
    sa.axp = hh.d_axp;
    sa.nseg = L.nseg;
    sa.r = r;
    sa.skip_topk = 1;
    HIPCHK(launch_select(&hh, sa, s));
    if (rrn) {
        hipLaunchKernelGGL(k_rrn_out, dim3(1), dim3(1), 0, s, (const Ctrl *)hh.d_ctrl, rrn);
        HIPCHK(hipGetLastError());
    }
    return RORBK_OK;
}
