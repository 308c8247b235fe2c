// Approximate distinguishing prefixes by prefix doubling (Section 4; proof
// outline in Appendix C) with exact duplicate detection: hash each active
// string's l-prefix, sort (hash, index) pairs, and a neighbour scan finds the
// duplicates (the local form of Appendix B's sorting-based detection).
#include "common.hpp"
#include "sort_core.hpp"

#define KR_P 0x1FFFFFFFFFFFFFFFull  // 2^61 - 1
#define KR_B 0x0B3C4D5E6F708192ull  // base

// a*b mod 2^61-1 for a, b < 2^61, using 2^64 = 8 (mod p).
__device__ __forceinline__ u64 mulmod61(u64 a, u64 b)
{
    const u64 lo = a * b;
    const u64 hi = __umul64hi(a, b);  // < 2^58
    u64 r = (lo & KR_P) + (lo >> 61) + (hi << 3);
    r = (r & KR_P) + (r >> 61);
    return r >= KR_P ? r - KR_P : r;
}

__device__ __forceinline__ u64 addmod61(u64 a, u64 b)
{
    u64 r = a + b;  // a < p, b < 2^33
    return r >= KR_P ? r - KR_P : r;
}

// Extend the Horner state C over bytes [from, m) of the string at `o` (from is
// a multiple of 4; limbs are 4-byte little-endian, the last zero-padded).
__device__ __forceinline__ u64 kr_extend(const u8 *bytes, u64 N, u64 o, u64 from, u64 m, u64 C)
{
    for (u64 q = from; q < m; q += 8) {
        const u64 r = m - q;
        const u32 take = r < 8 ? (u32)r : 8u;
        const u64 w = load_le(bytes, N, o + q, take);
        C = addmod61(mulmod61(C, KR_B), w & 0xFFFFFFFFull);
        if (take > 4) C = addmod61(mulmod61(C, KR_B), w >> 32);
    }
    return C;
}

__device__ __forceinline__ u64 kr_finish(u64 C, u64 m, u32 bits)
{
    u64 key = addmod61(mulmod61(C, KR_B), m);
    return bits >= 64 ? key : (key & ((1ull << bits) - 1));
}

__global__ __launch_bounds__(256) void k_prefix_keys(const u8 *bytes, u64 N, const u64 *off, u32 n,
                                                     u64 m, u32 bits, u64 *keys)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u64 o = off[i], len = off[i + 1] - o;
    const u64 mm = m < len ? m : len;
    keys[i] = kr_finish(kr_extend(bytes, N, o, 0, mm, 0), mm, bits);
}

struct BPow {
    u64 p[17];  // B^0 .. B^16 mod p
};

// One doubling round: key of the min(l, len)-prefix of every active string,
// continuing the Horner state of the previous round (bytes [lprev, l) only).
// A group of HG lanes (1, 2, 4 or 8, matched to the new bytes of the round)
// reads 8*HG consecutive bytes of one string per step; lane j folds its two
// limbs, and the group combines them as
// C <- C * B^L + sum_j v_j * B^(limbs after lane j).
template <int HG>
__global__ __launch_bounds__(256) void k_hash_round(const u32 *act, u32 A, const u8 *bytes, u64 N,
                                                    const u64 *off, u64 lprev, u64 l, u32 bits,
                                                    u64 *state, u64 *keys, u32 *vals, BPow bp)
{
    const u32 g = threadIdx.x / HG, lane = threadIdx.x % HG;
    const u32 j = blockIdx.x * (256 / HG) + g;
    if (j >= A) return;  // whole group leaves together
    const u32 i = act ? act[j] : j;
    const u64 o = off[i], len = off[i + 1] - o;
    const u64 m = l < len ? l : len;
    u64 C = lprev ? state[i] : 0ull;
    for (u64 x = lprev; x < m; x += 8 * HG) {
        const u64 q = x + 8 * lane;
        const u32 take = q < m ? (u32)((m - q) < 8 ? (m - q) : 8) : 0u;
        const u64 w = load_le(bytes, N, o + q, take);
        const u32 nl = take == 0 ? 0u : (take > 4 ? 2u : 1u);
        u64 v = 0;
        if (nl == 2) v = addmod61(mulmod61(w & 0xFFFFFFFFull, KR_B), w >> 32);
        else if (nl == 1) v = w & 0xFFFFFFFFull;
        const u64 rem = m - x;
        const u32 Lstep = (u32)((rem >= 8 * HG ? 8 * HG : rem) + 3) / 4;
        const u32 before = 2 * lane < Lstep ? 2 * lane : Lstep;
        const u32 after = Lstep - before - nl;
        u64 t = nl ? (after ? mulmod61(v, bp.p[after]) : v) : 0ull;
#pragma unroll
        for (int s2 = HG / 2; s2 > 0; s2 >>= 1) t = addmod61(t, __shfl_xor(t, s2, HG));
        C = addmod61(mulmod61(C, bp.p[Lstep]), t);
    }
    if (lane == 0) {
        state[i] = C;
        keys[j] = kr_finish(C, m, bits);
        vals[j] = j;  // position in the active list (kept in input order)
    }
}

#define PRE_MAX 64  // the first pass hashes up to this many bytes of every string
#define PRE_SLOTS 8

struct PreLens {
    u64 l[PRE_SLOTS];  // prefix lengths of the precomputed rounds (l_0, 2 l_0, ...)
    u32 count;
};

// First pass: a group of 8 lanes reads the first min(len, W) bytes of one
// string once (W = the last precomputed prefix length <= 64; lane j holds
// bytes [8j, 8j+8), i.e. limbs 2j and 2j+1) and emits the key of every round
// whose prefix length is <= W, by input index.  For a prefix of L limbs,
// C = sum_j (limb_2j*B + limb_2j+1) * B^(L-2-2j) over lanes with both limbs in
// the prefix, plus limb_2j for the lane whose second limb is past the prefix.
// Keys of later rounds continue from the Horner state of the W-prefix.
__global__ __launch_bounds__(256) void k_hash_first(u32 n, const u8 *bytes, u64 N, const u64 *off, PreLens P,
                                                    u32 bits, BPow bp, u64 *state, u64 *pre)
{
    const u32 lane = threadIdx.x & 7;
    const u32 i = blockIdx.x * 32 + (threadIdx.x >> 3);
    if (i >= n) return;  // whole group leaves together
    const u64 o = off[i], len = off[i + 1] - o;
    const u64 W = P.l[P.count - 1];
    const u64 mw = len < W ? len : W;
    const u64 q = 8ull * lane;
    const u32 take = q < mw ? (u32)((mw - q) < 8 ? (mw - q) : 8) : 0u;
    const u64 w = load_le(bytes, N, o + q, take);
    const u64 a = w & 0xFFFFFFFFull, b = w >> 32;
    const u64 v = addmod61(mulmod61(a, KR_B), b);
    u64 C = 0;
    for (u32 r = 0; r < P.count; r++) {
        const u64 m = len < P.l[r] ? len : P.l[r];
        const u32 L = (u32)((m + 3) / 4);
        u64 c = 0;
        if (2 * lane + 1 < L) c = mulmod61(v, bp.p[L - 2 - 2 * lane]);
        else if (2 * lane + 1 == L) c = a;
#pragma unroll
        for (int s2 = 4; s2 > 0; s2 >>= 1) c = addmod61(c, __shfl_xor(c, s2, 8));
        C = c;
        if (lane == 0) pre[(u64)r * n + i] = kr_finish(c, m, bits);
    }
    if (lane == 0) state[i] = C;
}

// Keys of a precomputed round for the active list (payload = list position).
__global__ __launch_bounds__(256) void k_gather_keys(const u32 *act, u32 A, const u64 *pre_r, u64 *keys, u32 *vals)
{
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A) return;
    keys[j] = pre_r[act ? act[j] : j];
    vals[j] = j;
}

__device__ __forceinline__ u64 lanemask_lt_h() { return (1ull << __lane_id()) - 1ull; }

// Finish strings whose key is unique among the active ones or whose length is
// <= l; the others are flagged (by their position in the active list) to stay.
__global__ __launch_bounds__(256) void k_dedup(const u64 *keys, const u32 *vals, u32 A, const u32 *act,
                                               const u64 *off, u64 l, u32 *dist, u32 *keep)
{
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A) return;
    const u64 k = keys[j];
    const bool dup = (j > 0 && keys[j - 1] == k) || (j + 1 < A && keys[j + 1] == k);
    const u32 p = vals[j];
    const u32 i = act ? act[p] : p;
    const u64 len = off[i + 1] - off[i];
    const bool stay = dup && len > l;
    if (!stay) dist[i] = (u32)(len < l ? len : l);
    keep[p] = stay ? 1u : 0u;
}

// Ordered compaction of the active list by the keep flags (pos = exclusive scan).
__global__ void k_compact(const u32 *act, u32 A, const u32 *keep, const u32 *pos, u32 *next)
{
    const u32 p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < A && keep[p]) next[pos[p]] = act ? act[p] : p;
}

__global__ void k_one_seg(Seg *act, u32 A) { act[0] = Seg{0, A, 0, 0}; }

// flag = 1 if some key differs from keys[0] (then the keys must be sorted)
__global__ void k_neq(const u64 *keys, u32 A, u32 *flag)
{
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < A && keys[j] != keys[0]) *flag = 1u;
}

struct PdWs {
    SortWs sw;
    u32 *vals, *actA, *actB, *ctr, *keep, *kpos;
    u64 *state, *pre, *scan_scratch;
};

static void pd_layout(u64 n, PdWs *w, WsArena *a, WsCounter *c)
{
    sort_ws_layout(n, &w->sw, a, c);
#define PT(field, T, cnt)                       \
    do {                                         \
        if (a) w->field = a->take<T>(cnt);       \
        else c->take<T>(cnt);                    \
    } while (0)
    PT(vals, u32, n); PT(actA, u32, n); PT(actB, u32, n); PT(state, u64, n); PT(ctr, u32, 4);
    PT(keep, u32, n); PT(kpos, u32, n + 1); PT(scan_scratch, u64, ss_scan_scratch_elems<u64>(n + 1));
    PT(pre, u64, (u64)PRE_SLOTS * n);
#undef PT
}

extern "C" size_t ss_dist_prefix_workspace(uint64_t n)
{
    WsCounter c;
    PdWs w;
    pd_layout(n, &w, nullptr, &c);
    return c.used;
}

extern "C" int ss_prefix_keys(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                              uint32_t m, uint32_t hash_bits, uint64_t *keys, void *stream)
{
    ss_clear_error();
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (hash_bits < 1 || hash_bits > 64) { ss_set_error("hash_bits must be 1..64"); return SS_ERR_INVALID_ARG; }
    if (n == 0) return SS_OK;
    if (!offsets || !keys) { ss_set_error("null pointer"); return SS_ERR_INVALID_ARG; }
    hipStream_t st = (hipStream_t)stream;
    k_prefix_keys<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(bytes, N, offsets, (u32)n, (u64)m, hash_bits,
                                                               keys);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

extern "C" int ss_dist_prefix(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                              uint32_t init_len, uint32_t hash_bits, uint32_t *dist_approx,
                              uint32_t *rounds_host, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (init_len == 0 || (init_len % 4) != 0) {
        ss_set_error("init_len must be a positive multiple of 4");
        return SS_ERR_INVALID_ARG;
    }
    if (hash_bits < 8 || hash_bits > 64) { ss_set_error("hash_bits must be 8..64"); return SS_ERR_INVALID_ARG; }
    if (rounds_host) *rounds_host = 0;
    if (n == 0) return SS_OK;
    if (!offsets || !dist_approx) { ss_set_error("null pointer"); return SS_ERR_INVALID_ARG; }
    hipStream_t st = (hipStream_t)stream;
    WsArena a(ws, ws_bytes);
    PdWs w;
    pd_layout(n, &w, &a, nullptr);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_dist_prefix_workspace(n));
        return SS_ERR_WORKSPACE;
    }
    BPow bp;
    bp.p[0] = 1;
    for (int t = 1; t <= 16; t++) bp.p[t] = (u64)(((unsigned __int128)bp.p[t - 1] * KR_B) % KR_P);
    // rounds whose prefix length is at most PRE_MAX are hashed in one first pass
    PreLens P{};
    for (u64 L = init_len; L <= PRE_MAX && P.count < PRE_SLOTS; L *= 2) P.l[P.count++] = L;
    if (P.count) {
        // the first line of every string, once
        SS_PROF("k_hash_first", st, (double)n * (double)P.l[P.count - 1] + (double)n * (24.0 + 8.0 * P.count));
        k_hash_first<<<(unsigned)ceil_div(n, 32), 256, 0, st>>>((u32)n, bytes, N, offsets, P, hash_bits, bp, w.state,
                                                                 w.pre);
    }
    SS_CHECK_LAUNCH();
    u32 A = (u32)n;
    const u32 *act = nullptr;  // the active strings, in input order (NULL = all)
    u32 *nxt = w.actA;
    u64 lprev = 0, l = init_len;
    u32 rounds = 0;
    while (A > 0) {
        if (++rounds > 64) { ss_set_error("prefix doubling did not terminate"); return SS_ERR_INVALID_ARG; }
        if (rounds <= P.count) {
            k_gather_keys<<<(unsigned)ceil_div(A, 256), 256, 0, st>>>(act, A, w.pre + (u64)(rounds - 1) * n,
                                                                      w.sw.keyA, w.vals);
            SS_CHECK_LAUNCH();
        } else {
            // new prefix bytes (exact for strings of length >= l), offsets, list entry,
            // hash state in/out, key and payload out
            SS_PROF("k_hash_round", st, (double)A * (double)(l - lprev) + (double)A * 48.0);
            const u64 nb = l - lprev;
            if (nb <= 8)
                k_hash_round<1><<<(unsigned)ceil_div(A, 256), 256, 0, st>>>(act, A, bytes, N, offsets, lprev, l,
                                                                           hash_bits, w.state, w.sw.keyA, w.vals, bp);
            else if (nb <= 16)
                k_hash_round<2><<<(unsigned)ceil_div(A, 128), 256, 0, st>>>(act, A, bytes, N, offsets, lprev, l,
                                                                           hash_bits, w.state, w.sw.keyA, w.vals, bp);
            else if (nb <= 32)
                k_hash_round<4><<<(unsigned)ceil_div(A, 64), 256, 0, st>>>(act, A, bytes, N, offsets, lprev, l,
                                                                          hash_bits, w.state, w.sw.keyA, w.vals, bp);
            else
                k_hash_round<8><<<(unsigned)ceil_div(A, 32), 256, 0, st>>>(act, A, bytes, N, offsets, lprev, l,
                                                                          hash_bits, w.state, w.sw.keyA, w.vals, bp);
        }
        SS_CHECK_LAUNCH();
        if (A >= 2) {
            // all keys equal (e.g. a prefix shared by every string): every
            // string is a duplicate and no sort is needed
            SS_HIP(hipMemsetAsync(w.ctr + 1, 0, sizeof(u32), st));
            k_neq<<<(unsigned)ceil_div(A, 256), 256, 0, st>>>(w.sw.keyA, A, w.ctr + 1);
            SS_CHECK_LAUNCH();
            u32 differ;
            SS_TRY(ss_read_u32(w.ctr + 1, &differ, 1, st));
            if (differ) {
                k_one_seg<<<1, 1, 0, st>>>(w.sw.act, A);
                SS_CHECK_LAUNCH();
                SortJob J{bytes, N, offsets, w.vals, nullptr, 1, st, A};
                SS_TRY(sort_rounds(J, w.sw, 1, (u32)ceil_div(A, 2048)));
            }
        }
        {
            SS_PROF("k_dedup", st, (double)A * 40.0);  // key, payload, list entry, offsets, one write
            k_dedup<<<(unsigned)ceil_div(A, 256), 256, 0, st>>>(w.sw.keyA, w.vals, A, act, offsets, l, dist_approx,
                                                                w.keep);
        }
        SS_CHECK_LAUNCH();
        SS_TRY(ss_scan_exclusive<u32>(w.keep, w.kpos, A, (u32 *)w.scan_scratch, st));
        k_compact<<<(unsigned)ceil_div(A, 256), 256, 0, st>>>(act, A, w.keep, w.kpos, nxt);
        SS_CHECK_LAUNCH();
        SS_TRY(ss_read_u32(w.kpos + A, &A, 1, st));
        act = nxt;
        nxt = (nxt == w.actA) ? w.actB : w.actA;
        lprev = l;
        l *= 2;
    }
    if (rounds_host) *rounds_host = rounds;
    return SS_OK;
}
