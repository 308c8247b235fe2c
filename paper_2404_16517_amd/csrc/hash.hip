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

// One doubling round: key of the min(l, len)-prefix of every active string,
// continuing the Horner state of the previous round (bytes [lprev, l) only).
__global__ __launch_bounds__(256) void k_hash_round(const u32 *act, u32 A, const u8 *bytes, u64 N,
                                                    const u64 *off, u64 lprev, u64 l, u32 bits,
                                                    u64 *state, u64 *keys, u32 *vals)
{
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A) return;
    const u32 i = act ? act[j] : j;
    const u64 o = off[i], len = off[i + 1] - o;
    const u64 m = l < len ? l : len;
    u64 C = lprev ? state[i] : 0ull;
    C = kr_extend(bytes, N, o, lprev, m, C);
    state[i] = C;
    keys[j] = kr_finish(C, m, bits);
    vals[j] = i;
}

__device__ __forceinline__ u64 lanemask_lt_h() { return (1ull << __lane_id()) - 1ull; }

// Finish strings whose key is unique among the active ones or whose length is
// <= l; the rest form the next active list.
__global__ __launch_bounds__(256) void k_dedup(const u64 *keys, const u32 *vals, u32 A, const u64 *off,
                                               u64 l, u32 *dist, u32 *next, u32 *ctr)
{
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = j < A;
    bool keep = false;
    u32 i = 0;
    if (valid) {
        const u64 k = keys[j];
        const bool dup = (j > 0 && keys[j - 1] == k) || (j + 1 < A && keys[j + 1] == k);
        i = vals[j];
        const u64 len = off[i + 1] - off[i];
        if (!dup || len <= l) dist[i] = (u32)(len < l ? len : l);
        else keep = true;
    }
    const u64 m = __ballot(keep);
    if (m == 0) return;
    const u32 leader = __ffsll((unsigned long long)m) - 1;
    u32 base = 0;
    if (__lane_id() == leader) base = atomicAdd(ctr, (u32)__popcll(m));
    base = __shfl(base, leader, 64);
    if (keep) next[base + (u32)__popcll(m & lanemask_lt_h())] = i;
}

__global__ void k_one_seg(Seg *act, u32 A) { act[0] = Seg{0, A, 0, 0}; }

struct PdWs {
    SortWs sw;
    u32 *vals, *actA, *actB, *ctr;
    u64 *state;
};

static void pd_layout(u64 n, PdWs *w, WsArena *a, WsCounter *c)
{
    sort_ws_layout(n, &w->sw, a, c);
    if (a) {
        w->vals = a->take<u32>(n);
        w->actA = a->take<u32>(n);
        w->actB = a->take<u32>(n);
        w->state = a->take<u64>(n);
        w->ctr = a->take<u32>(4);
    } else {
        c->take<u32>(n);
        c->take<u32>(n);
        c->take<u32>(n);
        c->take<u64>(n);
        c->take<u32>(4);
    }
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
    u32 A = (u32)n;
    const u32 *act = nullptr;
    u32 *nxt = w.actA;
    u64 lprev = 0, l = init_len;
    u32 rounds = 0;
    while (A > 0) {
        if (++rounds > 64) { ss_set_error("prefix doubling did not terminate"); return SS_ERR_INVALID_ARG; }
        k_hash_round<<<(unsigned)ceil_div(A, 256), 256, 0, st>>>(act, A, bytes, N, offsets, lprev, l, hash_bits,
                                                                  w.state, w.sw.keyA, w.vals);
        SS_CHECK_LAUNCH();
        if (A >= 2) {
            k_one_seg<<<1, 1, 0, st>>>(w.sw.act, A);
            SS_CHECK_LAUNCH();
            SortJob J{bytes, N, offsets, w.vals, nullptr, 1, st};
            SS_TRY(sort_rounds(J, w.sw, 1));
        }
        SS_HIP(hipMemsetAsync(w.ctr, 0, sizeof(u32), st));
        k_dedup<<<(unsigned)ceil_div(A, 256), 256, 0, st>>>(w.sw.keyA, w.vals, A, offsets, l, dist_approx, nxt,
                                                             w.ctr);
        SS_CHECK_LAUNCH();
        SS_TRY(ss_read_u32(w.ctr, &A, 1, st));
        act = nxt;
        nxt = (nxt == w.actA) ? w.actB : w.actA;
        lprev = l;
        l *= 2;
    }
    if (rounds_host) *rounds_host = rounds;
    return SS_OK;
}
