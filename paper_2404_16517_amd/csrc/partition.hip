// Splitters, bucket boundaries and LCP compression of buckets (Section 3,
// steps 1-2; LCP compression from Section 2; distinguishing prefixes only in
// the prefix-doubling variant of Section 4).
#include <string.h>

#include "common.hpp"

// ------------------------------------------------------------- splitters

// f_j = s_perm[ceil(j n / r) - 1], j = 1..r-1 (regular sampling of the whole
// sorted array, the one-device form of Section 3.1).
__global__ void k_select(u64 n, const u32 *perm, u32 r, u32 *ids)
{
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (j >= r) return;
    const u64 c = ((u64)j * n + r - 1) / r;
    ids[j - 1] = perm[c - 1];
}

extern "C" int ss_select_splitters(uint64_t n, const uint32_t *perm, uint32_t r, uint32_t *splitter_ids,
                                   void *stream)
{
    ss_clear_error();
    if (n == 0 || r == 0 || !perm || (r > 1 && !splitter_ids)) {
        ss_set_error("select_splitters needs n >= 1, r >= 1 and non-null arrays");
        return SS_ERR_INVALID_ARG;
    }
    if (r == 1) return SS_OK;
    hipStream_t st = (hipStream_t)stream;
    k_select<<<(unsigned)ceil_div(r - 1, 256), 256, 0, st>>>(n, perm, r, splitter_ids);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

// The same sampling applied to every set b of a batch (set b = positions
// [set_off[b], set_off[b+1]) of perm): one thread per (set, j).  Thread j = 1
// of each set also checks that the set is non-empty and well placed; a bad set
// raises *bad and its samples are written as 0xFFFFFFFF without reading perm.
__global__ void k_select_batch(const u32 *perm, u64 n, const u64 *set_off, u32 num_sets, u32 r, u32 *ids,
                               u32 *bad)
{
    const u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u32 per = r - 1;
    if (t >= (u64)num_sets * per) return;
    const u32 b = (u32)(t / per);
    const u32 j = (u32)(t - (u64)b * per) + 1;
    const u64 lo = set_off[b], hi = set_off[b + 1];
    const bool ok = lo < hi && hi <= n;
    if (bad && j == 1 && (!ok || (b == 0 && lo != 0) || (b == num_sets - 1 && hi != n))) atomicOr(bad, 1u);
    u32 v = 0xFFFFFFFFu;
    if (ok) {
        const u64 m = hi - lo;
        v = perm[lo + ((u64)j * m + r - 1) / r - 1];
    }
    ids[t] = v;
}

extern "C" size_t ss_select_splitters_batch_workspace(void) { return 256; }

extern "C" int ss_select_splitters_batch(const uint32_t *perm, uint64_t n, const uint64_t *set_off,
                                         uint32_t num_sets, uint32_t r, uint32_t *splitter_ids, void *ws,
                                         size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (n == 0 || r == 0 || num_sets == 0 || !perm || !set_off || (r > 1 && !splitter_ids)) {
        ss_set_error("select_splitters_batch needs n >= 1, r >= 1, num_sets >= 1 and non-null arrays");
        return SS_ERR_INVALID_ARG;
    }
    if ((u64)num_sets * (r - 1) >= 0xFFFFFFFFull) {
        ss_set_error("num_sets * (r - 1) too large");
        return SS_ERR_TOO_LARGE;
    }
    if (r == 1) return SS_OK;
    hipStream_t st = (hipStream_t)stream;
    const u64 total = (u64)num_sets * (r - 1);
    if (!ws && ws_bytes == 0) {  // unchecked: nothing read back
        k_select_batch<<<(unsigned)ceil_div(total, 256), 256, 0, st>>>(perm, n, set_off, num_sets, r, splitter_ids,
                                                                       nullptr);
        SS_CHECK_LAUNCH();
        return SS_OK;
    }
    if (!ws || ws_bytes < sizeof(u32)) {
        ss_set_error("workspace too small: need %zu bytes", ss_select_splitters_batch_workspace());
        return SS_ERR_WORKSPACE;
    }
    u32 *bad = (u32 *)ws;
    SS_HIP(hipMemsetAsync(bad, 0, sizeof(u32), st));
    k_select_batch<<<(unsigned)ceil_div(total, 256), 256, 0, st>>>(perm, n, set_off, num_sets, r, splitter_ids,
                                                                   bad);
    SS_CHECK_LAUNCH();
    u32 h;
    SS_TRY(ss_read_u32(bad, &h, 1, st));
    if (h) {
        ss_set_error("every set must be non-empty, with set_off[0] = 0, set_off[num_sets] = n and "
                     "set_off increasing");
        return SS_ERR_INVALID_ARG;
    }
    return SS_OK;
}

// ----------------------------------------------- character-based splitters
//
// Character-based regular sampling (Section 3.1, Appendix A): equally spaced
// positions of each sorted set's character array, each shifted back to the
// start of the string holding it.  P[i] = characters of the strings at sorted
// positions < i (all sets in one scan); in set b = [lo, hi) with N_b =
// P[hi] - P[lo], sample j (1..r-1) is at x = P[lo] + ceil(j N_b / r) - 1 and
// picks the largest position k in [lo, hi) with P[k] <= x (empty strings share
// P with the next string, so the pick always holds x); N_b = 0 picks lo.

__global__ void k_char_counts(const u32 *perm, const u64 *off, const u32 *w, u64 n, u64 *P)
{
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32 s = perm[i];
    P[i] = w ? (u64)w[s] : off[s + 1] - off[s];
}

__global__ void k_select_chars_batch(const u32 *perm, const u64 *P, u64 n, const u64 *set_off, u32 num_sets,
                                     u32 r, u32 *ids, u32 *bad)
{
    const u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    const u32 per = r - 1;
    if (t >= (u64)num_sets * per) return;
    const u32 b = (u32)(t / per);
    const u32 j = (u32)(t - (u64)b * per) + 1;
    const u64 lo = set_off[b], hi = set_off[b + 1];
    const bool ok = lo < hi && hi <= n;
    if (bad && j == 1 && (!ok || (b == 0 && lo != 0) || (b == num_sets - 1 && hi != n))) atomicOr(bad, 1u);
    u32 v = 0xFFFFFFFFu;
    if (ok) {
        const u64 base = P[lo], Nb = P[hi] - base;
        u64 k = lo;
        if (Nb > 0) {
            const u64 x = base + ((u64)j * Nb + r - 1) / r - 1;
            u64 a = lo, e = hi;  // largest k in [a, e) with P[k] <= x (P[lo] <= x holds)
            while (e - a > 1) {
                const u64 m = (a + e) >> 1;
                if (P[m] <= x) a = m;
                else e = m;
            }
            k = a;
        }
        v = perm[k];
    }
    ids[t] = v;
}

extern "C" size_t ss_select_splitters_chars_batch_workspace(uint64_t n)
{
    WsCounter c;
    c.take<u64>(n + 1);
    c.take<u64>(ss_scan_scratch_elems<u64>(n + 1));
    c.take<u32>(1);
    return c.used;
}

extern "C" int ss_select_splitters_chars_batch(const uint32_t *perm, const uint64_t *offsets, const uint32_t *weights,
                                               uint64_t n, const uint64_t *set_off, uint32_t num_sets, uint32_t r,
                                               uint32_t *splitter_ids, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (n == 0 || r == 0 || num_sets == 0 || !perm || !offsets || !set_off || (r > 1 && !splitter_ids)) {
        ss_set_error("select_splitters_chars_batch needs n >= 1, r >= 1, num_sets >= 1 and non-null arrays");
        return SS_ERR_INVALID_ARG;
    }
    if (n >= 0xFFFFFFFFull || (u64)num_sets * (r - 1) >= 0xFFFFFFFFull) {
        ss_set_error("n or num_sets * (r - 1) too large");
        return SS_ERR_TOO_LARGE;
    }
    if (r == 1) return SS_OK;
    WsArena a(ws, ws_bytes);
    u64 *P = a.take<u64>(n + 1);
    u64 *scratch = a.take<u64>(ss_scan_scratch_elems<u64>(n + 1));
    u32 *bad = a.take<u32>(1);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_select_splitters_chars_batch_workspace(n));
        return SS_ERR_WORKSPACE;
    }
    hipStream_t st = (hipStream_t)stream;
    k_char_counts<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(perm, offsets, weights, n, P);
    SS_CHECK_LAUNCH();
    SS_TRY(ss_scan_exclusive<u64>(P, P, n, scratch, st));
    SS_HIP(hipMemsetAsync(bad, 0, sizeof(u32), st));
    const u64 total = (u64)num_sets * (r - 1);
    k_select_chars_batch<<<(unsigned)ceil_div(total, 256), 256, 0, st>>>(perm, P, n, set_off, num_sets, r,
                                                                         splitter_ids, bad);
    SS_CHECK_LAUNCH();
    u32 h;
    SS_TRY(ss_read_u32(bad, &h, 1, st));
    if (h) {
        ss_set_error("every set must be non-empty, with set_off[0] = 0, set_off[num_sets] = n and "
                     "set_off increasing");
        return SS_ERR_INVALID_ARG;
    }
    return SS_OK;
}

// ---------------------------------------------------------------- gather

// (an id >= n -- e.g. the UINT32_MAX sample of a malformed set -- is an empty string)
__global__ void k_gather_lens(const u64 *off, u64 n, const u32 *ids, u32 m, u64 *out)
{
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) out[j] = ids[j] < n ? off[ids[j] + 1] - off[ids[j]] : 0ull;
}

// one wave per string, lanes copy consecutive bytes; a string ending past cap
// is not copied (the caller that read nothing back sees out_off[m] > cap)
__global__ __launch_bounds__(256) void k_gather_copy(const u8 *bytes, const u64 *off, u64 n, const u32 *ids,
                                                     u32 m, const u64 *out_off, u8 *out, u64 cap)
{
    const u32 j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= m || ids[j] >= n) return;
    const u32 lane = threadIdx.x & 63;
    const u64 so = off[ids[j]], len = off[ids[j] + 1] - so, oo = out_off[j];
    if (oo + len > cap) return;
    for (u64 q = lane; q < len; q += 64) out[oo + q] = bytes[so + q];
}

extern "C" size_t ss_gather_workspace(uint64_t m)
{
    WsCounter c;
    c.take<u64>(ss_scan_scratch_elems<u64>(m + 1));
    return c.used;
}

extern "C" int ss_gather_strings(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                 const uint32_t *ids, uint64_t m, uint64_t *out_offsets, uint8_t *out_bytes,
                                 uint64_t out_cap, uint64_t *total_host, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    (void)N;
    if (m >= 0xFFFFFFFFull) { ss_set_error("m too large"); return SS_ERR_TOO_LARGE; }
    if (!out_offsets || (m > 0 && (!offsets || !ids))) { ss_set_error("null pointer"); return SS_ERR_INVALID_ARG; }
    hipStream_t st = (hipStream_t)stream;
    WsArena a(ws, ws_bytes);
    u64 *scratch = a.take<u64>(ss_scan_scratch_elems<u64>(m + 1));
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_gather_workspace(m));
        return SS_ERR_WORKSPACE;
    }
    if (m > 0) {
        k_gather_lens<<<(unsigned)ceil_div(m, 256), 256, 0, st>>>(offsets, n, ids, (u32)m, out_offsets);
        SS_CHECK_LAUNCH();
    }
    SS_TRY(ss_scan_exclusive<u64>(out_offsets, out_offsets, m, scratch, st));
    if (!total_host) {  // nothing read back: the copy checks the capacity per string
        if (m > 0) {
            k_gather_copy<<<(unsigned)ceil_div(m, 4), 256, 0, st>>>(bytes, offsets, n, ids, (u32)m, out_offsets,
                                                                    out_bytes, out_cap);
            SS_CHECK_LAUNCH();
        }
        return SS_OK;
    }
    u64 total;
    SS_TRY(ss_read_u64(out_offsets + m, &total, 1, st));
    if (total_host) *total_host = total;
    if (total > out_cap) {
        ss_set_error("gather needs %llu bytes, capacity %llu", (unsigned long long)total,
                     (unsigned long long)out_cap);
        return SS_ERR_CAPACITY;
    }
    if (m > 0 && total > 0) {
        k_gather_copy<<<(unsigned)ceil_div(m, 4), 256, 0, st>>>(bytes, offsets, n, ids, (u32)m, out_offsets,
                                                                out_bytes, out_cap);
        SS_CHECK_LAUNCH();
    }
    return SS_OK;
}

// --------------------------------------------------------------- buckets

// bounds of set b: run_off[b*(r+1) + j] = set_off[b] + #{ s in set b : s <= f_j }
// (set_off == NULL: one set [0, n)).  One wavefront per bound: a 9-ary search
// whose eight pivots per step are compared with f by eight lanes each (64
// bytes per round, from the LCP that the interval's ends share with f).
__global__ __launch_bounds__(256) void k_bounds(const u8 *bytes, u64 N, const u64 *off, const u64 *set_off, u64 n,
                                                u32 nsets, const u32 *perm, const u8 *sb, u64 sN, const u64 *soff,
                                                u32 r, u64 *bounds)
{
    const u64 t = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const u32 lane = threadIdx.x & 63, grp = lane >> 3, gl = lane & 7;
    if (t >= (u64)nsets * (r + 1)) return;  // uniform over the wavefront
    const u32 b = (u32)(t / (r + 1)), j = (u32)(t % (r + 1));
    u64 lo = set_off ? set_off[b] : 0, hi = set_off ? set_off[b + 1] : n;
    if (j == 0 || j == r) {
        if (lane == 0) bounds[t] = j == 0 ? lo : hi;
        return;
    }
    const u64 fo = soff[j - 1], fl = soff[j] - fo;
    u64 llo = 0, lhi = 0;  // LCPs of f with the strings just outside [lo, hi)
    while (lo < hi) {      // uniform over the wavefront
        const u64 len = hi - lo;
        const u32 np = len < 8 ? (u32)len : 8u;
        const bool act = grp < np;
        const u64 piv = len < 8 ? lo + grp : lo + ((u64)(grp + 1) * len) / 9;  // increasing in grp
        u64 o = 0, l = 0;
        if (act) {
            const u32 p = perm[piv];
            o = off[p];
            l = off[p + 1] - o;
        }
        const u64 m = l < fl ? l : fl;
        u64 pos = llo < lhi ? llo : lhi;
        int cmp = 0;
        u64 lc = 0;
        bool done = !act;
        while (__ballot(!done)) {  // 64-byte rounds until every group has decided
            u64 mis = ~0ull;
            int sgn = 0;
            if (!done) {
                const u64 q = pos + 8ull * gl;
                const u32 take = q < m ? (m - q < 8 ? (u32)(m - q) : 8u) : 0u;
                if (take) {
                    const u64 wa = load_be(bytes, N, o + q, take), wb = load_be(sb, sN, fo + q, take);
                    if (wa != wb) {
                        mis = q + (__clzll(wa ^ wb) >> 3);
                        sgn = wa < wb ? -1 : 1;
                    }
                }
            }
            // the group's first mismatch and its sign (the lowest lane that has one)
#pragma unroll
            for (u32 d = 1; d < 8; d <<= 1) {
                const u64 m2 = __shfl_xor(mis, d, 8);
                const int s2 = __shfl_xor(sgn, d, 8);
                if (m2 < mis) {
                    mis = m2;
                    sgn = s2;
                }
            }
            if (!done) {
                if (mis != ~0ull) {
                    lc = mis;
                    cmp = sgn;
                    done = true;
                } else if (pos + 64 >= m) {  // equal up to the shorter length
                    lc = m;
                    cmp = l < fl ? -1 : (l > fl ? 1 : 0);
                    done = true;
                } else {
                    pos += 64;
                }
            }
        }
        // the first pivot above f: the interval between it and the one before
        const u64 above = __ballot(act && gl == 0 && cmp > 0);
        const u32 g = above ? (u32)(__builtin_ctzll(above) >> 3) : np;
        const u64 pg = __shfl(piv, 8 * (g < np ? g : 0)), lg = __shfl(lc, 8 * (g < np ? g : 0));
        const u64 pb = __shfl(piv, 8 * (g ? g - 1 : 0)), lb = __shfl(lc, 8 * (g ? g - 1 : 0));
        if (g < np) {
            hi = pg;
            lhi = lg;
        }
        if (g > 0) {
            lo = pb + 1;
            llo = lb;
        }
    }
    if (lane == 0) bounds[t] = lo;
}

extern "C" int ss_bucket_bounds(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                const uint32_t *perm, const uint8_t *spl_bytes, uint64_t spl_N,
                                const uint64_t *spl_offsets, uint32_t r, uint64_t *bounds, void *stream)
{
    ss_clear_error();
    if (r == 0 || !bounds || (r > 1 && !spl_offsets) || (n > 0 && (!offsets || !perm))) {
        ss_set_error("bucket_bounds: bad arguments");
        return SS_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    k_bounds<<<(unsigned)ceil_div((u64)r + 1, 4), 256, 0, st>>>(bytes, N, offsets, nullptr, n, 1, perm, spl_bytes,
                                                                spl_N, spl_offsets, r, bounds);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

// ---------------------------------------------------------- front coding

// e_i, d_i, id_i and the literal length d_i - e_i of every sorted position.
// run_off holds nb = sets*(r+1) non-decreasing bucket bounds (the bounds of
// all sets, one after the other); position i starts a bucket iff some bound
// equals i, and otherwise the largest bound below i is its bucket's start.
__global__ __launch_bounds__(256) void k_fc_meta(const u64 *off, u32 n, const u32 *perm, const u32 *lcp,
                                                 const u32 *dist, const u64 *run_off, u32 nb, u32 *fc_lcp,
                                                 u32 *fc_len, u32 *fc_id, u64 *sizes, u64 *lit_src, u32 *bad)
{
    // bucket start: the largest run_off[j] <= i.  The workgroup's positions
    // are contiguous: one search for its first position, then each thread
    // steps forward over the (few) bucket bounds inside the workgroup.
    __shared__ u32 s_lo;
    const u32 i0 = blockIdx.x * blockDim.x;
    if (threadIdx.x == 0) {
        u32 lo = 0, hi = nb - 1;
        while (hi - lo > 1) {
            u32 mid = (lo + hi) >> 1;
            if (run_off[mid] <= i0) lo = mid;
            else hi = mid;
        }
        s_lo = lo;
    }
    __syncthreads();
    const u32 i = i0 + threadIdx.x;
    if (i >= n) return;
    u32 lo = s_lo;
    while (lo + 2 < nb && run_off[lo + 1] <= i) lo++;
    const u32 e = (run_off[lo] == i) ? 0u : lcp[i];
    const u32 p = perm[i];
    const u64 o = off[p], len = off[p + 1] - o;
    const u32 d = dist ? dist[p] : (u32)len;
    fc_lcp[i] = e;
    fc_len[i] = d;
    fc_id[i] = p;
    lit_src[i] = o + e;  // where the literal starts, in sorted order for the copy
    if (e > d || d > len) {
        atomicOr(bad, 1u);
        sizes[i] = 0;
    } else {
        sizes[i] = d - e;
    }
}

__global__ void k_add_base(u64 *a, u64 n, u64 base)
{
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += base;
}

#define CS_NT 256     // strings per workgroup in the literal copy (one thread each)
#define CS_BUF 4096   // LDS staging bytes (short literals: at most 16 B per string on average)

// Literal bytes of strings [i0, i0+256) (string i's bytes [e_i, d_i) go to
// suf[suf_off[i] ..]; lit_src[i] = offset of byte e_i, written in sorted order
// by k_fc_meta).  When the workgroup's output span fits the LDS buffer (short
// literals, as distinguishing prefixes of D/N strings leave them) each
// thread reads its string's literal with aligned 8-byte words, the literals
// are packed in LDS and written out in aligned 16-byte words (bytes at the
// two ends, which neighbouring workgroups share, one by one).  Otherwise
// (longer literals, where one thread's word loop and byte stores cost more
// than idle lanes) 4, 8 or 16 lanes, by the workgroup's average literal, copy
// one string at a time: every lane an aligned 8-byte word of the destination,
// read from the source at whatever alignment it has, and the unaligned bytes
// at the two ends one by one.
__global__ __launch_bounds__(CS_NT) void k_fc_copy(const u8 *bytes, u64 N, u32 n, const u64 *lit_src,
                                                   const u64 *suf_off, u8 *suf)
{
    __shared__ uint4 buf4[CS_BUF / 16];
    u8 *buf = (u8 *)buf4;
    const u32 i0 = blockIdx.x * CS_NT;
    const u32 i1 = (i0 + CS_NT < n) ? i0 + CS_NT : n;
    const u64 S0 = suf_off[i0], S1 = suf_off[i1];
    const u64 span = S1 - S0;
    const u32 mis = (u32)(((uintptr_t)(suf + S0)) & 15);  // buf[mis] holds output byte S0
    const bool staged = span + mis <= CS_BUF;
    if (!staged) {  // uniform over the workgroup
        // lanes per string by the workgroup's average literal: 4 up to 48
        // bytes, 8 up to 128, else 16
        const u64 avg = span / (i1 - i0);
        const u32 lsh = avg <= 48 ? 2u : (avg <= 128 ? 3u : 4u), L = 1u << lsh;
        const u32 gl = threadIdx.x & (L - 1);
        for (u32 i = i0 + (threadIdx.x >> lsh); i < i1; i += CS_NT >> lsh) {
            const u64 so = suf_off[i], len = suf_off[i + 1] - so, src = lit_src[i];
            const u32 mis8 = (u32)(((uintptr_t)(suf + so)) & 7);
            const u64 head = mis8 ? (8u - mis8 < len ? 8u - mis8 : len) : 0u;  // bytes up to an aligned word
            const u64 words = (len - head) / 8;
            for (u64 t = gl; t < head; t += L) suf[so + t] = bytes[src + t];
            for (u64 q = gl; q < words; q += L)
                *(u64 *)(suf + so + head + 8 * q) = load_le(bytes, N, src + head + 8 * q, 8u);
            for (u64 t = head + 8 * words + gl; t < len; t += L) suf[so + t] = bytes[src + t];
        }
        return;
    }
    const u32 i = i0 + threadIdx.x;
    if (i < i1) {
        const u64 so = suf_off[i], len = suf_off[i + 1] - so;
        const u64 src = lit_src[i];
        for (u64 k = 0; k < len; k += 8) {
            const u32 take = (len - k) < 8 ? (u32)(len - k) : 8u;
            const u64 w = load_le(bytes, N, src + k, take);
            const u64 b = so - S0 + mis + k;
            for (u32 t = 0; t < take; t++) buf[b + t] = (u8)(w >> (8 * t));
        }
    }
    __syncthreads();
    const u32 nchunk = (u32)((span + mis + 15) / 16);
    for (u32 c = threadIdx.x; c < nchunk; c += CS_NT) {
        const u64 r = 16ull * c;  // buffer offset of the chunk; output byte S0 - mis + r
        if (r >= mis && r + 16 - mis <= span) {
            *(uint4 *)(suf + (S0 + r - mis)) = buf4[c];
        } else {
            for (u32 t = 0; t < 16; t++) {
                const u64 q = r + t;
                if (q >= mis && q - mis < span) suf[S0 + q - mis] = buf[q];
            }
        }
    }
}

extern "C" size_t ss_partition_encode_workspace(uint64_t n)
{
    WsCounter c;
    c.take<u64>(ss_scan_scratch_elems<u64>(n + 1));
    c.take<u32>(4);
    c.take<u64>(n);  // literal source offsets
    return c.used;
}

__global__ void k_put_u64(u64 *dst, const u64 *src) { *dst = *src; }

static int encode_impl(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n, const uint64_t *set_off,
                       uint32_t nsets, const uint32_t *perm, const uint32_t *lcp, const uint32_t *dist,
                       const uint8_t *spl_bytes, uint64_t spl_N, const uint64_t *spl_offsets, uint32_t r,
                       uint64_t *run_off, uint32_t *fc_lcp, uint32_t *fc_len, uint32_t *fc_id, uint64_t *suf_off,
                       uint8_t *suf, uint64_t suf_base, uint64_t suf_cap, uint64_t *suf_total_host, void *ws,
                       size_t ws_bytes, void *stream)
{
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (r == 0 || nsets == 0 || !run_off || !suf_off || (r > 1 && !spl_offsets) ||
        (n > 0 && (!offsets || !perm || !lcp || !fc_lcp || !fc_len || !fc_id))) {
        ss_set_error("partition_encode: bad arguments");
        return SS_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    WsArena a(ws, ws_bytes);
    u64 *scratch = a.take<u64>(ss_scan_scratch_elems<u64>(n + 1));
    u32 *bad = a.take<u32>(4);
    u64 *lit_src = a.take<u64>(n);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_partition_encode_workspace(n));
        return SS_ERR_WORKSPACE;
    }
    const u64 nb = (u64)nsets * (r + 1);
    k_bounds<<<(unsigned)ceil_div(nb, 4), 256, 0, st>>>(bytes, N, offsets, set_off, n, nsets, perm, spl_bytes,
                                                        spl_N, spl_offsets, r, run_off);
    SS_CHECK_LAUNCH();
    SS_HIP(hipMemsetAsync(bad, 0, sizeof(u32), st));
    if (n > 0) {
        {
            // perm, lcp, offsets, dist in; e, d, id, the literal length and source out
            SS_PROF("k_fc_meta", st, (double)n * (dist ? 56.0 : 52.0));
            k_fc_meta<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(offsets, (u32)n, perm, lcp, dist, run_off, (u32)nb,
                                                                   fc_lcp, fc_len, fc_id, suf_off, lit_src, bad);
        }
        SS_CHECK_LAUNCH();
    }
    SS_TRY(ss_scan_exclusive<u64>(suf_off, suf_off, n, scratch, st));
    if (suf_base) {
        k_add_base<<<(unsigned)ceil_div(n + 1, 256), 256, 0, st>>>(suf_off, n + 1, suf_base);
        SS_CHECK_LAUNCH();
    }
    // the check flag and the literal total side by side, one read-back
    k_put_u64<<<1, 1, 0, st>>>((u64 *)(bad + 2), suf_off + n);
    SS_CHECK_LAUNCH();
    u32 hw[4];
    SS_TRY(ss_read_u32(bad, hw, 4, st));
    const u32 hbad = hw[0];
    u64 total;
    memcpy(&total, hw + 2, sizeof(u64));
    total -= suf_base;
    if (hbad) {
        ss_set_error("front coding needs lcp <= dist <= len at every position");
        return SS_ERR_INVALID_ARG;
    }
    if (suf_base + total > suf_cap) {
        ss_set_error("literal bytes %llu exceed capacity %llu", (unsigned long long)(suf_base + total),
                     (unsigned long long)suf_cap);
        return SS_ERR_CAPACITY;
    }
    if (suf_total_host) *suf_total_host = total;
    if (total > 0) {
        {
            // literal bytes read and written; per string its perm, offsets, e and suf_off
            SS_PROF("k_fc_copy", st, 2.0 * (double)total + (double)n * 16.0);
            k_fc_copy<<<(unsigned)ceil_div(n, CS_NT), CS_NT, 0, st>>>(bytes, N, (u32)n, lit_src, suf_off, suf);
        }
        SS_CHECK_LAUNCH();
    }
    return SS_OK;
}

extern "C" int ss_partition_encode(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                   const uint32_t *perm, const uint32_t *lcp, const uint32_t *dist,
                                   const uint8_t *spl_bytes, uint64_t spl_N, const uint64_t *spl_offsets,
                                   uint32_t r, uint64_t *run_off, uint32_t *fc_lcp, uint32_t *fc_len,
                                   uint32_t *fc_id, uint64_t *suf_off, uint8_t *suf, uint64_t suf_base,
                                   uint64_t suf_cap, uint64_t *suf_total_host, void *ws, size_t ws_bytes,
                                   void *stream)
{
    ss_clear_error();
    return encode_impl(bytes, N, offsets, n, nullptr, 1, perm, lcp, dist, spl_bytes, spl_N, spl_offsets, r, run_off,
                       fc_lcp, fc_len, fc_id, suf_off, suf, suf_base, suf_cap, suf_total_host, ws, ws_bytes, stream);
}

extern "C" int ss_partition_encode_batch(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                         const uint64_t *set_off, uint32_t num_sets, const uint32_t *perm,
                                         const uint32_t *lcp, const uint32_t *dist, const uint8_t *spl_bytes,
                                         uint64_t spl_N, const uint64_t *spl_offsets, uint32_t r, uint64_t *run_off,
                                         uint32_t *fc_lcp, uint32_t *fc_len, uint32_t *fc_id, uint64_t *suf_off,
                                         uint8_t *suf, uint64_t suf_base, uint64_t suf_cap,
                                         uint64_t *suf_total_host, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (!set_off || num_sets == 0) {
        ss_set_error("partition_encode_batch needs set_off and num_sets >= 1");
        return SS_ERR_INVALID_ARG;
    }
    return encode_impl(bytes, N, offsets, n, set_off, num_sets, perm, lcp, dist, spl_bytes, spl_N, spl_offsets, r,
                       run_off, fc_lcp, fc_len, fc_id, suf_off, suf, suf_base, suf_cap, suf_total_host, ws,
                       ws_bytes, stream);
}
