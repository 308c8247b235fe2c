// Suffix sorting as repeated sorting of equal-length strings (the paper's
// Section 6 names suffix sorting based on sorting strings of equal length as
// the next application), space-efficiently: the suffixes T[i, N) overlap and
// are never stored.  Prefix doubling over ranks: rank_h(i) is the rank of
// suffix i's h-character prefix among all such prefixes; the 2h-prefix of
// suffix i is the pair (rank_h(i), rank_h(i + h)) (rank 0 past the text), so
// each step sorts N equal-length strings -- the pairs written as W big-endian
// bytes -- with the library's string sort and re-ranks from it, until every
// rank is distinct.  The first step sorts the first K bytes of every suffix
// followed by its remaining length capped at K (so that a suffix ending
// inside the window sorts before its extensions, whatever bytes follow).
#include "common.hpp"

#define SFX_K 6  // first step: K bytes + one length byte = 7-byte strings

// Ranks are < 2^28 when N < 2^28: a pair fits 56 bits = 7 bytes (one sort
// round of 7-byte keys); otherwise 32 + 32 bits in 8 bytes.
struct SfxShape {
    u32 W;     // bytes per string
    u32 bits;  // bits per rank
};

static SfxShape sfx_shape(u64 N) { return N < (1ull << 28) ? SfxShape{7, 28} : SfxShape{8, 32}; }

__device__ __forceinline__ void put_be(u8 *dst, u64 v, u32 W)
{
    for (u32 b = 0; b < W; b++) dst[b] = (u8)(v >> (8 * (W - 1 - b)));
}

// First step: string i = T[i, i+K) zero-padded, then min(K, N - i); its value
// (the same order) is kept as a word for the re-ranking.
__global__ void k_sfx_init(const u8 *T, u64 N, u8 *keys, u32 W, u64 *val, u64 *koff)
{
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    koff[i] = i * W;
    if (i == N) return;
    const u64 rem = N - i;
    const u32 take = rem < SFX_K ? (u32)rem : SFX_K;
    u64 v = load_be(T, N, i, take) >> (8 * (8 - SFX_K));  // K bytes, zero-padded
    v = (v << 8) | take;
    val[i] = v;
    u8 *d = keys + i * W;
    for (u32 b = 0; b < W; b++) d[b] = b + 7 < W ? 0 : (u8)(v >> (8 * (W - 1 - b)));
}

// Doubling step: string i = (rank(i), rank(i + h)) as W big-endian bytes.
__global__ void k_sfx_pairs(const u32 *rank, u64 N, u64 h, u32 bits, u32 W, u8 *keys, u64 *val)
{
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const u64 r2 = i + h < N ? rank[i + h] : 0u;
    const u64 v = ((u64)rank[i] << bits) | r2;
    val[i] = v;
    put_be(keys + i * W, v, W);
}

// flag[k] = 1 where the sorted value changes (k = 0 included).
__global__ void k_sfx_flags(const u32 *sa, const u64 *val, u64 N, u32 *flag)
{
    const u64 k = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    flag[k] = (k == 0 || val[sa[k]] != val[sa[k - 1]]) ? 1u : 0u;
}

// rank(sa[k]) = number of distinct values up to sorted position k (>= 1).
__global__ void k_sfx_rank(const u32 *sa, const u32 *excl, const u32 *flag, u64 N, u32 *rank)
{
    const u64 k = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    rank[sa[k]] = excl[k] + flag[k];
}

// lcp[k] = lcp of the suffixes at sorted positions k-1 and k, by comparing
// 8 bytes at a time (cost: the sum of the LCPs, the suffixes' D).
__global__ void k_sfx_lcp(const u8 *T, u64 N, const u32 *sa, u32 *lcp)
{
    const u64 k = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    if (k == 0) {
        lcp[0] = 0;
        return;
    }
    const u64 a = sa[k - 1], b = sa[k];
    const u64 m = N - (a > b ? a : b);
    u64 l = 0;
    while (l < m) {
        const u32 take = (m - l) < 8 ? (u32)(m - l) : 8u;
        const u64 x = load_be(T, N, a + l, take), y = load_be(T, N, b + l, take);
        if (x != y) {
            l += __clzll(x ^ y) >> 3;
            break;
        }
        l += take;
    }
    lcp[k] = (u32)l;
}

struct SfxWs {
    u8 *keys;
    u64 *koff, *val;
    u32 *rank, *flag, *excl, *scan_scratch;
    void *sort_ws;
    size_t sort_bytes;
};

static void sfx_layout(u64 N, SfxWs *w, WsArena *a, WsCounter *c)
{
    const SfxShape sh = sfx_shape(N);
    const size_t sort_bytes = ss_sort_workspace(N);
#define TK(field, T, cnt)                      \
    do {                                        \
        if (a) w->field = a->take<T>(cnt);      \
        else c->take<T>(cnt);                   \
    } while (0)
    TK(keys, u8, N * sh.W);
    TK(koff, u64, N + 1);
    TK(val, u64, N);
    TK(rank, u32, N);
    TK(flag, u32, N);
    TK(excl, u32, N + 1);
    TK(scan_scratch, u32, ss_scan_scratch_elems<u32>(N + 1));
#undef TK
    if (a) {
        w->sort_ws = a->take<u8>(sort_bytes);
        w->sort_bytes = sort_bytes;
    } else {
        c->take<u8>(sort_bytes);
    }
}

extern "C" size_t ss_suffix_sort_workspace(uint64_t N)
{
    WsCounter c;
    SfxWs w;
    sfx_layout(N, &w, nullptr, &c);
    return c.used;
}

extern "C" int ss_suffix_sort(const uint8_t *text, uint64_t N, uint32_t *sa, uint32_t *lcp, uint32_t *steps_host,
                              void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (steps_host) *steps_host = 0;
    if (N >= 0xFFFFFFFFull) {
        ss_set_error("text of %llu bytes beyond the 32-bit index limit", (unsigned long long)N);
        return SS_ERR_TOO_LARGE;
    }
    if (N == 0) return SS_OK;
    if (!text || !sa) {
        ss_set_error("null text or sa");
        return SS_ERR_INVALID_ARG;
    }
    WsArena a(ws, ws_bytes);
    SfxWs w;
    sfx_layout(N, &w, &a, nullptr);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_suffix_sort_workspace(N));
        return SS_ERR_WORKSPACE;
    }
    hipStream_t st = (hipStream_t)stream;
    const SfxShape sh = sfx_shape(N);
    const unsigned g = (unsigned)ceil_div(N + 1, 256);
    k_sfx_init<<<g, 256, 0, st>>>(text, N, w.keys, sh.W, w.val, w.koff);
    SS_CHECK_LAUNCH();
    u64 h = SFX_K;
    u32 steps = 0;
    for (;;) {
        steps++;
        // sort the N equal-length strings of this step, then re-rank
        SS_TRY(ss_sort(w.keys, N * sh.W, w.koff, N, sa, nullptr, w.sort_ws, w.sort_bytes, stream));
        k_sfx_flags<<<g, 256, 0, st>>>(sa, w.val, N, w.flag);
        SS_CHECK_LAUNCH();
        SS_TRY(ss_scan_exclusive<u32>(w.flag, w.excl, N, w.scan_scratch, st));
        k_sfx_rank<<<g, 256, 0, st>>>(sa, w.excl, w.flag, N, w.rank);
        SS_CHECK_LAUNCH();
        u32 distinct = 0;
        SS_TRY(ss_read_u32(w.excl + N, &distinct, 1, st));
        if (distinct == N || h >= N) break;
        k_sfx_pairs<<<g, 256, 0, st>>>(w.rank, N, h, sh.bits, sh.W, w.keys, w.val);
        SS_CHECK_LAUNCH();
        h *= 2;
    }
    if (lcp) {
        k_sfx_lcp<<<g, 256, 0, st>>>(text, N, sa, lcp);
        SS_CHECK_LAUNCH();
    }
    if (steps_host) *steps_host = steps;
    return SS_OK;
}
