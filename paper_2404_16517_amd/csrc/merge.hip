// Front-coding decode and LCP-aware k-way merge of sorted runs (Section 3,
// step 3; the LCP-aware merge building block of Section 2).
//
// Decode.  Within a run, string i equals the first e_i bytes of string i-1
// followed by its literal.  Its bytes [e_i, d_i) are its own literal; bytes
// [e_j, e_i) with j = psv(i) = the nearest earlier position with e_j < e_i are
// string j's literal, and so on down the psv chain to an e = 0 position (every
// run starts with e = 0).  psv is found first inside 256-element blocks (LDS),
// then by skipping blocks and 65536-element superblocks whose minimum is not
// smaller.  Each output 16-byte word then walks the chain of its string.
//
// Merge.  The paper merges r runs with an LCP loser tree.  Here the runs are
// merged pairwise in log2 k levels; each level is split into fixed-size output
// ranges by merge-path co-ranking, and every thread merges its range with the
// LCP rule: with h_a = lcp(last, a) and h_b = lcp(last, b), the larger of h_a,
// h_b decides without touching characters, and only on equality are the
// strings compared from h on.
#include <string.h>

#include <vector>

#include "common.hpp"

#define DB 256      // psv block
#define DSB 65536   // psv superblock

// ---------------------------------------------------------------- decode

__global__ __launch_bounds__(256) void k_check_runs(const u64 *run_off, u32 k, const u32 *e, const u32 *d,
                                                    u32 n, u32 *bad)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (run_off[0] != 0 || run_off[k] != n)) atomicOr(bad, 1u);
    if (i < k) {
        const u64 s = run_off[i];
        if (run_off[i + 1] < s || run_off[i + 1] > n) atomicOr(bad, 1u);
        else if (run_off[i + 1] > s && e[s] != 0) atomicOr(bad, 2u);
    }
    if (i < n) {
        if (e[i] > d[i]) atomicOr(bad, 4u);
        if (i > 0 && e[i] > d[i - 1]) atomicOr(bad, 4u);
    }
}

__global__ __launch_bounds__(DB) void k_psv_block(const u32 *e, u32 n, u32 *psv, u32 *bmin)
{
    __shared__ u32 se[DB];
    const u32 b0 = blockIdx.x * DB;
    const u32 i = b0 + threadIdx.x;
    const u32 v = i < n ? e[i] : 0xFFFFFFFFu;
    se[threadIdx.x] = v;
    __syncthreads();
    if (i < n) {
        u32 res = 0xFFFFFFFFu;  // not found in block
        if (v > 0) {
            for (int j = (int)threadIdx.x - 1; j >= 0; j--) {
                if (se[j] < v) { res = b0 + (u32)j; break; }
            }
        }
        psv[i] = res;
    }
    // block minimum
    u32 m = v;
    for (int o = 32; o > 0; o >>= 1) { u32 y = __shfl_xor(m, o, 64); m = y < m ? y : m; }
    __shared__ u32 wm[DB / 64];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 r = wm[0];
        for (int w = 1; w < DB / 64; w++) r = wm[w] < r ? wm[w] : r;
        bmin[blockIdx.x] = r;
    }
}

__global__ void k_min_reduce(const u32 *in, u32 nin, u32 group, u32 *out)
{
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    const u32 a = j * group;
    if (a >= nin) return;
    u32 m = 0xFFFFFFFFu;
    for (u32 t = a; t < a + group && t < nin; t++) m = in[t] < m ? in[t] : m;
    out[j] = m;
}

// psv for positions whose answer lies before their block.
__global__ __launch_bounds__(256) void k_psv_far(const u32 *e, u32 n, const u32 *bmin, const u32 *smin,
                                                 u32 *psv)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32 v = e[i];
    if (v == 0 || psv[i] != 0xFFFFFFFFu) return;
    const u32 blk = i / DB;
    const u32 per = DSB / DB;
    int b = (int)blk - 1;
    // blocks of the own superblock
    const int sb_first = (int)(blk / per) * (int)per;
    while (b >= sb_first && bmin[b] >= v) b--;
    if (b < sb_first) {
        int s = (int)(blk / per) - 1;
        while (s >= 0 && smin[s] >= v) s--;
        if (s < 0) { psv[i] = 0xFFFFFFFFu; return; }  // malformed input (no e = 0 before)
        b = s * (int)per + (int)per - 1;
        while (bmin[b] >= v) b--;
    }
    int j = b * DB + DB - 1;
    if (j > (int)n - 1) j = (int)n - 1;
    while (e[j] >= v) j--;
    psv[i] = (u32)j;
}

#define DC_NT 256
#define DC_PER 16

// Decoded bytes, 16 per thread, in output order.
__global__ __launch_bounds__(DC_NT) void k_decode(const u32 *e, const u32 *d, const u64 *suf_off,
                                                  const u8 *suf, const u32 *psv, u32 n, const u64 *out_off,
                                                  u64 total, u8 *out)
{
    __shared__ u32 range[2];
    const u64 c0 = (u64)blockIdx.x * DC_NT * DC_PER;
    const u64 c1 = (c0 + DC_NT * DC_PER < total) ? c0 + DC_NT * DC_PER : total;
    if (threadIdx.x < 2) {
        const u64 q = threadIdx.x == 0 ? c0 : c1 - 1;
        u32 lo = 0, hi = n;
        while (hi - lo > 1) {
            u32 mid = (lo + hi) >> 1;
            if (out_off[mid] <= q) lo = mid;
            else hi = mid;
        }
        range[threadIdx.x] = lo;
    }
    __syncthreads();
    const u64 q0 = c0 + (u64)threadIdx.x * DC_PER;
    if (q0 >= c1) return;
    u32 lo = range[0], hi = range[1] + 1;
    while (hi - lo > 1) {
        u32 mid = (lo + hi) >> 1;
        if (out_off[mid] <= q0) lo = mid;
        else hi = mid;
    }
    u32 i = lo;
    u64 so = out_off[i], se = out_off[i + 1];
    const u32 cnt = (u32)((c1 - q0) < DC_PER ? (c1 - q0) : DC_PER);
    u8 buf[DC_PER];
    u32 pj = 0, plo = 1, phi = 0;  // current piece: string pj covers bytes [plo, phi)
#pragma unroll
    for (u32 t = 0; t < DC_PER; t++) {
        if (t < cnt) {
            const u64 q = q0 + t;
            while (q >= se) {
                i++;
                so = se;
                se = out_off[i + 1];
                plo = 1; phi = 0;
            }
            const u32 kk = (u32)(q - so);
            if (kk < plo || kk >= phi) {
                u32 j = i, h = d[i];
                while (e[j] > kk) { h = e[j]; j = psv[j]; }
                pj = j; plo = e[j]; phi = h;
            }
            buf[t] = suf[suf_off[pj] + (kk - plo)];
        } else {
            buf[t] = 0;
        }
    }
    u8 *dst = out + q0;
    if (cnt == DC_PER && (((uintptr_t)dst) & 15) == 0) {
        uint4 v;
        v.x = buf[0] | (buf[1] << 8) | (buf[2] << 16) | ((u32)buf[3] << 24);
        v.y = buf[4] | (buf[5] << 8) | (buf[6] << 16) | ((u32)buf[7] << 24);
        v.z = buf[8] | (buf[9] << 8) | (buf[10] << 16) | ((u32)buf[11] << 24);
        v.w = buf[12] | (buf[13] << 8) | (buf[14] << 16) | ((u32)buf[15] << 24);
        *(uint4 *)dst = v;
    } else {
        for (u32 t = 0; t < cnt; t++) dst[t] = buf[t];
    }
}

__global__ void k_widen(const u32 *d, u32 n, u64 *out)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = d[i];
}

struct DecWs {
    u32 *psv, *bmin, *smin, *bad;
    u64 *scratch;
};

static void dec_layout(u64 n, DecWs *w, WsArena *a, WsCounter *c)
{
    const u64 nb = n / DB + 2, ns = n / DSB + 2;
    if (a) {
        w->psv = a->take<u32>(n + 1);
        w->bmin = a->take<u32>(nb);
        w->smin = a->take<u32>(ns);
        w->bad = a->take<u32>(4);
        w->scratch = a->take<u64>(ss_scan_scratch_elems<u64>(n + 1));
    } else {
        c->take<u32>(n + 1);
        c->take<u32>(nb);
        c->take<u32>(ns);
        c->take<u32>(4);
        c->take<u64>(ss_scan_scratch_elems<u64>(n + 1));
    }
}

static int decode_impl(u32 k, const u64 *run_off, const u32 *e, const u32 *d, const u64 *suf_off, const u8 *suf,
                       u64 n, u64 *out_off, u8 *out, u64 out_cap, DecWs &w, hipStream_t st)
{
    SS_HIP(hipMemsetAsync(w.bad, 0, sizeof(u32), st));
    const u64 grid = ceil_div((n > k ? n : k) + 1, 256);
    k_check_runs<<<(unsigned)grid, 256, 0, st>>>(run_off, k, e, d, (u32)n, w.bad);
    SS_CHECK_LAUNCH();
    if (n > 0) {
        k_widen<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(d, (u32)n, out_off);
        SS_CHECK_LAUNCH();
    }
    SS_TRY(ss_scan_exclusive<u64>(out_off, out_off, n, w.scratch, st));
    u32 bad;
    u64 total;
    SS_TRY(ss_read_u32(w.bad, &bad, 1, st));
    SS_TRY(ss_read_u64(out_off + n, &total, 1, st));
    if (bad) {
        ss_set_error("malformed front-coded runs (code %u): runs must start with e = 0 and e_i <= d_i, "
                     "e_i <= d_{i-1}", bad);
        return SS_ERR_INVALID_ARG;
    }
    if (total > out_cap) {
        ss_set_error("decoded bytes %llu exceed capacity %llu", (unsigned long long)total,
                     (unsigned long long)out_cap);
        return SS_ERR_CAPACITY;
    }
    if (n == 0 || total == 0) return SS_OK;
    const u32 nb = (u32)ceil_div(n, DB);
    k_psv_block<<<nb, DB, 0, st>>>(e, (u32)n, w.psv, w.bmin);
    SS_CHECK_LAUNCH();
    const u32 per = DSB / DB;
    const u32 ns = (u32)ceil_div(nb, per);
    k_min_reduce<<<(unsigned)ceil_div(ns, 256), 256, 0, st>>>(w.bmin, nb, per, w.smin);
    SS_CHECK_LAUNCH();
    k_psv_far<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(e, (u32)n, w.bmin, w.smin, w.psv);
    SS_CHECK_LAUNCH();
    k_decode<<<(unsigned)ceil_div(total, DC_NT * DC_PER), DC_NT, 0, st>>>(e, d, suf_off, suf, w.psv, (u32)n, out_off,
                                                                       total, out);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

extern "C" size_t ss_fc_decode_workspace(uint64_t n)
{
    WsCounter c;
    DecWs w;
    dec_layout(n, &w, nullptr, &c);
    return c.used;
}

extern "C" int ss_fc_decode(uint32_t k, const uint64_t *run_off, const uint32_t *fc_lcp, const uint32_t *fc_len,
                            const uint64_t *suf_off, const uint8_t *suf, uint64_t n, uint64_t *out_offsets,
                            uint8_t *out_bytes, uint64_t out_cap, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (k == 0 || !run_off || !out_offsets || (n > 0 && (!fc_lcp || !fc_len || !suf_off))) {
        ss_set_error("fc_decode: bad arguments");
        return SS_ERR_INVALID_ARG;
    }
    WsArena a(ws, ws_bytes);
    DecWs w;
    dec_layout(n, &w, &a, nullptr);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_fc_decode_workspace(n));
        return SS_ERR_WORKSPACE;
    }
    return decode_impl(k, run_off, fc_lcp, fc_len, suf_off, suf, n, out_offsets, out_bytes, out_cap, w,
                       (hipStream_t)stream);
}

// ----------------------------------------------------------------- merge

#define MG_PER 32  // outputs per thread

struct MergeLevel {
    const u32 *G, *L;     // input element ids (decoded string index) and lcp
    u32 *Go, *Lo;         // outputs
    const u64 *R;         // run bounds of this level (device, nruns+1)
    const u32 *tstart;    // per pair: first thread (device, npairs+1)
    u32 npairs;
    u32 nruns;
    const u8 *db;         // decoded bytes
    u64 dN;
    const u64 *doff;      // decoded offsets
};

__device__ __forceinline__ int cmp_g(const MergeLevel &M, u32 x, u32 y, u64 from, u64 *lcp)
{
    const u64 ox = M.doff[x], lx = M.doff[x + 1] - ox;
    const u64 oy = M.doff[y], ly = M.doff[y + 1] - oy;
    return str_cmp_from(M.db, M.dN, ox, lx, M.db, M.dN, oy, ly, from, lcp);
}

__global__ __launch_bounds__(256) void k_merge_level(MergeLevel M, u32 nthreads)
{
    const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nthreads) return;
    // pair of this thread: largest p with tstart[p] <= t
    u32 lo = 0, hi = M.npairs;
    while (hi - lo > 1) {
        u32 mid = (lo + hi) >> 1;
        if (M.tstart[mid] <= t) lo = mid;
        else hi = mid;
    }
    const u32 p = lo;
    const u32 ra = 2 * p, rb = 2 * p + 1;
    const u64 A0 = M.R[ra], A1 = M.R[ra + 1];
    const u64 B0 = (rb < M.nruns) ? M.R[rb] : A1;
    const u64 B1 = (rb < M.nruns) ? M.R[rb + 1] : A1;
    const u32 na = (u32)(A1 - A0), nb = (u32)(B1 - B0);
    const u32 dloc = (t - M.tstart[p]) * MG_PER;
    const u32 tot = na + nb;
    if (dloc >= tot) return;
    const u32 cnt = (tot - dloc) < MG_PER ? (tot - dloc) : MG_PER;
    const u32 *GA = M.G + A0, *LA = M.L + A0, *GB = M.G + B0, *LB = M.L + B0;
    u64 tmp;
    // co-rank: x = number of A elements among the first dloc outputs
    u32 xlo = dloc > nb ? dloc - nb : 0, xhi = dloc < na ? dloc : na;
    while (xlo < xhi) {
        const u32 mid = (xlo + xhi) >> 1;
        // A[mid] <= B[dloc-mid-1] -> A[mid] is among the first dloc outputs
        if (cmp_g(M, GA[mid], GB[dloc - mid - 1], 0, &tmp) <= 0) xlo = mid + 1;
        else xhi = mid;
    }
    u32 a = xlo, b = dloc - xlo;
    // LCPs of the next candidates with the previous output
    u32 ha = 0, hb = 0;
    if (dloc > 0) {
        bool lastA;
        if (a == 0) lastA = false;
        else if (b == 0) lastA = true;
        else lastA = cmp_g(M, GA[a - 1], GB[b - 1], 0, &tmp) > 0;  // A[a-1] > B[b-1] -> A[a-1] was last
        if (lastA) {
            if (a < na) ha = LA[a];
            if (b < nb) { cmp_g(M, GA[a - 1], GB[b], 0, &tmp); hb = (u32)tmp; }
        } else {
            if (b < nb) hb = LB[b];
            if (a < na) { cmp_g(M, GB[b - 1], GA[a], 0, &tmp); ha = (u32)tmp; }
        }
    }
    u32 *Go = M.Go + A0 + dloc, *Lo = M.Lo + A0 + dloc;
    for (u32 k = 0; k < cnt; k++) {
        bool takeA;
        u32 outl;
        if (a >= na) {
            takeA = false;
            outl = hb;
        } else if (b >= nb) {
            takeA = true;
            outl = ha;
        } else if (ha > hb) {
            takeA = true;
            outl = ha;
        } else if (ha < hb) {
            takeA = false;
            outl = hb;
        } else {
            const int c = cmp_g(M, GA[a], GB[b], ha, &tmp);
            outl = ha;
            if (c <= 0) {
                takeA = true;
                hb = (u32)tmp;
            } else {
                takeA = false;
                ha = (u32)tmp;
            }
        }
        if (dloc + k == 0) outl = 0;
        if (takeA) {
            Go[k] = GA[a];
            Lo[k] = outl;
            a++;
            if (a < na) ha = LA[a];
        } else {
            Go[k] = GB[b];
            Lo[k] = outl;
            b++;
            if (b < nb) hb = LB[b];
        }
    }
}

__global__ void k_merge_init(const u32 *e, u32 n, u32 *G, u32 *L)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    G[i] = i;
    L[i] = e[i];
}

__global__ void k_merge_out(const u32 *G, const u32 *L, u32 n, const u64 *run_off, u32 k, const u32 *fc_id,
                            u64 *src, u32 *id, u32 *lcp)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32 g = G[i];
    u32 lo = 0, hi = k;  // largest run j with run_off[j] <= g
    while (hi - lo > 1) {
        u32 mid = (lo + hi) >> 1;
        if (run_off[mid] <= g) lo = mid;
        else hi = mid;
    }
    src[i] = ((u64)lo << 32) | (u64)(g - run_off[lo]);
    id[i] = fc_id[g];
    lcp[i] = i == 0 ? 0u : L[i];
}

struct MergeWs {
    DecWs dec;
    u64 *doff;
    u32 *G0, *G1, *L0, *L1;
    u64 *R;
    u32 *tstart;
};

// Fixed part of the merge workspace; the decoded bytes take the rest.
static void merge_layout(u64 n, u64 k, MergeWs *w, WsArena *a, WsCounter *c)
{
    dec_layout(n, &w->dec, a, c);
    if (a) {
        w->doff = a->take<u64>(n + 1);
        w->G0 = a->take<u32>(n);
        w->G1 = a->take<u32>(n);
        w->L0 = a->take<u32>(n);
        w->L1 = a->take<u32>(n);
        w->R = a->take<u64>(k + 2);
        w->tstart = a->take<u32>(k + 2);
    } else {
        c->take<u64>(n + 1);
        c->take<u32>(n);
        c->take<u32>(n);
        c->take<u32>(n);
        c->take<u32>(n);
        c->take<u64>(k + 2);
        c->take<u32>(k + 2);
    }
}

#define MERGE_MAX_K 65536

extern "C" size_t ss_lcp_merge_workspace(uint64_t n, uint64_t total_len)
{
    WsCounter c;
    MergeWs w;
    merge_layout(n, MERGE_MAX_K, &w, nullptr, &c);
    c.take<u8>(total_len + 16);
    return c.used;
}

extern "C" int ss_lcp_merge(uint32_t k, const uint64_t *run_off, const uint32_t *fc_lcp, const uint32_t *fc_len,
                            const uint32_t *fc_id, const uint64_t *suf_off, const uint8_t *suf, uint64_t n,
                            uint64_t *out_src, uint32_t *out_id, uint32_t *out_lcp, void *ws, size_t ws_bytes,
                            void *stream)
{
    ss_clear_error();
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (k == 0 || k > MERGE_MAX_K || !run_off || (n > 0 && (!fc_lcp || !fc_len || !fc_id || !suf_off || !out_src ||
                                                             !out_id || !out_lcp))) {
        ss_set_error("lcp_merge: bad arguments (1 <= k <= %d)", MERGE_MAX_K);
        return SS_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    std::vector<u64> R(k + 1);
    SS_HIP(hipMemcpyAsync(R.data(), run_off, sizeof(u64) * (k + 1), hipMemcpyDeviceToHost, st));
    SS_HIP(hipStreamSynchronize(st));
    if (R[0] != 0 || R[k] != n) {
        ss_set_error("run_off must start at 0 and end at n");
        return SS_ERR_INVALID_ARG;
    }
    WsArena a(ws, ws_bytes);
    MergeWs w;
    merge_layout(n, MERGE_MAX_K, &w, &a, nullptr);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes plus the decoded bytes", ss_lcp_merge_workspace(n, 0));
        return SS_ERR_WORKSPACE;
    }
    u8 *db = a.base + a.used;
    const u64 budget = ws_bytes - a.used;
    SS_TRY(decode_impl(k, run_off, fc_lcp, fc_len, suf_off, suf, n, w.doff, db, budget, w.dec, st));
    if (n == 0) return SS_OK;
    u64 dN;
    SS_TRY(ss_read_u64(w.doff + n, &dN, 1, st));
    k_merge_init<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(fc_lcp, (u32)n, w.G0, w.L0);
    SS_CHECK_LAUNCH();
    u32 *G = w.G0, *L = w.L0, *Go = w.G1, *Lo = w.L1;
    std::vector<u64> cur(R);
    std::vector<u32> ts;
    while (cur.size() - 1 > 1) {
        const u32 nr = (u32)(cur.size() - 1);
        const u32 np = (nr + 1) / 2;
        ts.assign(np + 1, 0);
        for (u32 p = 0; p < np; p++) {
            const u64 sz = cur[std::min<u64>(2 * p + 2, nr)] - cur[2 * p];
            ts[p + 1] = ts[p] + (u32)ceil_div(sz ? sz : 1, MG_PER);
        }
        SS_HIP(hipMemcpyAsync(w.R, cur.data(), sizeof(u64) * (nr + 1), hipMemcpyHostToDevice, st));
        SS_HIP(hipMemcpyAsync(w.tstart, ts.data(), sizeof(u32) * (np + 1), hipMemcpyHostToDevice, st));
        MergeLevel M{G, L, Go, Lo, w.R, w.tstart, np, nr, db, dN, w.doff};
        const u32 nth = ts[np];
        k_merge_level<<<(unsigned)ceil_div(nth, 256), 256, 0, st>>>(M, nth);
        SS_CHECK_LAUNCH();
        // the host vectors must stay valid until the copies ran
        SS_HIP(hipStreamSynchronize(st));
        std::vector<u64> nxt;
        for (u32 p = 0; p < np; p++) nxt.push_back(cur[2 * p]);
        nxt.push_back(cur[nr]);
        cur.swap(nxt);
        std::swap(G, Go);
        std::swap(L, Lo);
    }
    k_merge_out<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(G, L, (u32)n, run_off, k, fc_id, out_src, out_id,
                                                            out_lcp);
    SS_CHECK_LAUNCH();
    return SS_OK;
}
