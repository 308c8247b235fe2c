// Approximate distinguishing prefixes by prefix doubling (Section 4; proof
// outline in Appendix C) with exact duplicate detection: hash each active
// string's l-prefix and find the keys that occur more than once among the
// active strings.  The paper detects them by sorting (hash, index) pairs and
// scanning neighbours (Appendix B); on one GPU an open-addressing table of the
// keys gives the same multiplicities in two passes without the sort.
#include "common.hpp"

#define KR_P 0x1FFFFFFFFFFFFFFFull  // 2^61 - 1
#define KR_B 0x0B3C4D5E6F708192ull  // base

// a*b mod 2^61-1 for a, b < 2^61.  With 32-bit halves (a1, b1 < 2^29):
// a*b = a0 b0 + (a0 b1 + a1 b0) 2^32 + a1 b1 2^64, and 2^61 = 1, 2^64 = 8
// (mod p); the middle term times 2^32 folds as (mid mod 2^29) 2^32 + mid / 2^29.
__device__ __forceinline__ u64 mulmod61(u64 a, u64 b)
{
    const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    const u64 p00 = (u64)a0 * b0;
    const u64 mid = (u64)a0 * b1 + (u64)a1 * b0;  // < 2^62
    const u64 p11 = (u64)a1 * b1;                 // < 2^58
    u64 r = (p00 & KR_P) + (p00 >> 61) + ((mid & 0x1FFFFFFFull) << 32) + (mid >> 29) + (p11 << 3);
    r = (r & KR_P) + (r >> 61);
    return r >= KR_P ? r - KR_P : r;
}

// a*b mod 2^61-1 for a < 2^32, b < 2^61.
__device__ __forceinline__ u64 mulmod61_32(u32 a, u64 b)
{
    const u64 p00 = (u64)a * (u32)b;
    const u64 mid = (u64)a * (u32)(b >> 32);  // < 2^61
    u64 r = (p00 & KR_P) + (p00 >> 61) + ((mid & 0x1FFFFFFFull) << 32) + (mid >> 29);
    r = (r & KR_P) + (r >> 61);
    return r >= KR_P ? r - KR_P : r;
}

__device__ __forceinline__ u64 addmod61(u64 a, u64 b)
{
    u64 r = a + b;  // a < p, b < 2^33
    return r >= KR_P ? r - KR_P : r;
}

// The key of an m-byte prefix from its weighted byte sum G (see the first
// pass): the Horner value is H = B^L G (L limbs) and the key (H B + m) =
// G B^(L+1) + m, so one product with bl1 = B^(L+1).
__device__ __forceinline__ u64 kr_key(u64 G, u64 bl1, u64 m, u32 bits)
{
    u64 key = addmod61(mulmod61(G, bl1), m);
    return bits >= 64 ? key : (key & ((1ull << bits) - 1));
}

struct BPow {
    u64 p[32];  // B^0 .. B^31 mod p
};

#define PRE_MAX 64  // the first pass hashes up to this many bytes of every string
#define PRE_SLOTS 5  // 4, 8, 16, 32, 64
#define PRE_ALL (PRE_SLOTS + 2)  // and 128, 256 when the first pass reads deeper

struct PreLens {
    u64 l[PRE_ALL];  // prefix lengths of the precomputed rounds (l_0, 2 l_0, ...)
    u32 count;
};

// First pass as a matrix product.  With the byte weights
// w_i = 256^(i mod 4) B^-(i/4 + 1) (mod p), the m-byte prefix of a string has
// G = sum_{i<m} byte_i w_i and Horner value H = B^L G (L = ceil(m/4) limbs,
// the last zero-padded), the same value as limb-by-limb Horner.  Each weight
// is split into nine 7-bit digits, w_i = sum_d c_id 2^(7d), so that each
// digit sum is an int8 dot product of the prefix bytes with one digit column;
// the first pass evaluates them for every precomputed round at once on the
// 32x32x32 int8 MFMA (see the round kernel for the layout).
struct FirstW {
    u64 ib[16];  // B^-(j+1) mod p for limbs j < 16 (the first 64 bytes)
};

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u64 rot61(u64 x, u32 k)  // x 2^k mod 2^61-1, x < p, k < 61
{
    return k == 0 ? x : (((x << k) & KR_P) | (x >> (61 - k)));
}

__device__ __forceinline__ u64 modp_i32(int s) { return s >= 0 ? (u64)s : (u64)((long long)s + (long long)KR_P); }

// Bytes [a, a+take) (take <= 16) as two little-endian words, the rest zero;
// reads only inside [bytes, bytes + N).  Split in two so that callers can
// issue the loads of several windows before combining any: issue() loads the
// three aligned words around the window when all of them lie inside the
// buffer, finish() shifts them into place (or reads bytes one by one near the
// buffer's ends).
struct Win16 {
    u64 w0, w1, w2;
    u64 a;
    u32 take, sh;
    bool ok;
};

__device__ __forceinline__ Win16 win16_issue(const u8 *__restrict__ bytes, u64 N, u64 a, u32 take)
{
    Win16 r;
    r.a = a;
    r.take = take;
    const u8 *pb = bytes + a;
    r.sh = (u32)((uintptr_t)pb & 7);
    const u8 *base = pb - r.sh;  // aligned; derived from bytes, so a global-memory pointer
    r.ok = take > 0 && base >= bytes && base + 24 <= bytes + N;
    r.w0 = r.w1 = r.w2 = 0;
    if (r.ok) {
        const u64 *w = (const u64 *)base;
        r.w0 = w[0];
        r.w1 = w[1];
        r.w2 = w[2];
    }
    return r;
}

__device__ __forceinline__ void win16_finish(const u8 *__restrict__ bytes, const Win16 &r, u64 &lo, u64 &hi)
{
    lo = hi = 0;
    if (r.take == 0) return;
    if (r.ok) {
        if (r.sh == 0) {
            lo = r.w0;
            hi = r.w1;
        } else {
            lo = (r.w0 >> (8 * r.sh)) | (r.w1 << (64 - 8 * r.sh));
            hi = (r.w1 >> (8 * r.sh)) | (r.w2 << (64 - 8 * r.sh));
        }
    } else {
        for (u32 t = 0; t < r.take; t++) {
            const u64 v = (u64)bytes[r.a + t];
            if (t < 8) lo |= v << (8 * t);
            else hi |= v << (8 * (t - 8));
        }
    }
    if (r.take < 8) {
        lo &= (1ull << (8 * r.take)) - 1ull;
        hi = 0;
    } else if (r.take < 16) {
        hi &= r.take == 8 ? 0ull : ((1ull << (8 * (r.take - 8))) - 1ull);
    }
}

__device__ __forceinline__ void load16_le(const u8 *__restrict__ bytes, u64 N, u64 a, u32 take, u64 &lo, u64 &hi)
{
    win16_finish(bytes, win16_issue(bytes, N, a, take), lo, hi);
}

// Round flags, three words per round: [0] minimum key, [1] maximum key,
// [2] nonzero if some string is no longer than the round's prefix length.
// Initialised by k_flag_init; all keys are equal iff min == max.
// Minimum, maximum and or of the flags over each lane half (32 lanes).
__device__ __forceinline__ void flags_reduce32(u64 &mn, u64 &mx, u64 &sh)
{
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const u64 a = __shfl_xor(mn, d), b = __shfl_xor(mx, d), c = __shfl_xor(sh, d);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
        sh |= c;
    }
}

__device__ __forceinline__ void flags_commit(u64 *f, u64 mn, u64 mx, u64 sh)
{
    if (mn != ~0ull) atomicMin((unsigned long long *)&f[0], (unsigned long long)mn);
    if (mx != 0ull) atomicMax((unsigned long long *)&f[1], (unsigned long long)mx);
    if (sh) atomicOr((unsigned long long *)&f[2], 1ull);
}

__global__ void k_flag_init(u64 *f, u32 words, u32 zero_from)
{
    const u32 t = threadIdx.x;
    if (t < words) f[t] = (t % 3 == 0 && t < zero_from) ? ~0ull : 0ull;
}

// Whether the first pass should also precompute rounds 128 and 256: at least
// 90 % of up to 4096 evenly spaced strings are at least 128 bytes long and
// share their first 64 bytes with the first of them (e.g. strings with a
// long common prefix).  One thread per sampled string; *count (zeroed before)
// receives the number that qualify.  Only the amount of bytes read depends on
// the decision.
#define DEEP_SAMPLE 4096
__global__ __launch_bounds__(256) void k_deep_probe(u32 n, const u8 *bytes, u64 N, const u64 *off, u64 *count)
{
    const u32 S = n < DEEP_SAMPLE ? n : DEEP_SAMPLE;
    const u32 k = blockIdx.x * blockDim.x + threadIdx.x;
    bool same = false;
    if (k < S) {
        const u32 i = (u32)((u64)k * n / S);
        const u64 o0 = off[0], l0 = off[1] - o0;
        const u64 o = off[i], l = off[i + 1] - o;
        u64 a[8], b[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {  // every load first
            a[q] = l >= 64 ? load_le(bytes, N, o + 8 * q, 8) : 0ull;
            b[q] = l0 >= 64 ? load_le(bytes, N, o0 + 8 * q, 8) : 0ull;
        }
        same = l >= 128 && l0 >= 128;
#pragma unroll
        for (int q = 0; q < 8; q++) same = same && a[q] == b[q];
    }
    const u64 m = __ballot(same);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd((unsigned long long *)count, (unsigned long long)__popcll(m));
}

// The deep decision from the probe's count over the sample of n strings.
__device__ __host__ __forceinline__ bool deep_from_count(u64 count, u32 n)
{
    const u64 S = n < DEEP_SAMPLE ? n : DEEP_SAMPLE;
    return S > 0 && 10ull * count >= 9ull * S;
}

// Later rounds continue the same sum, G_l = G_lprev + sum_{lprev<=i<l} byte_i
// w_i, over a list of active strings.  Positions are taken in chunks of 1024
// bytes: inside chunk c, w_(1024c+P) = w_P B^(-256c), so one table of digit
// weights for P < 1024 (built in LDS by each workgroup) serves every chunk and
// the int32 sums of a chunk are scaled by B^(-256c) once.  Each byte is split
// as 128 h + low (h in {0,1}, low < 128) so that both MFMA operands are
// non-negative and bytes past the string (zero) add nothing.
//
// One v_mfma_i32_32x32x32_i8 takes 32 bytes of 32 strings (B operand: column =
// string, lane l holds string l mod 32, bytes 16 (l / 32) .. + 16 of the
// block) against 32 weight rows (A operand).  Lane l's results are rows
// 8 (r / 4) + 4 (l / 32) + r mod 4 of its string (r < 16): row set 0 (rows
// 0..3, 8..11, 16, 17) lands in registers 0..9 of lane half 0, row set 1
// (rows 4..7, 12..15, 20, 21) in registers 0..9 of half 1.  Set 0 holds the
// full weights, set 1 the weights below l1 (two-round launches).  Register d
// sums the products of the low bits with digit d and, from a second product
// whose weight rows are shifted by one, of the high bits with digit d - 1
// (128 c 2^(7(d-1)) = c 2^(7d)).  Every lane combines its own ten sums: half 0
// carries G to l_end, half 1 carries G to l1, with no exchange between lanes.
struct RoundW {
    u64 iblo[16];  // B^-(r+1), r < 16
    u64 ibhi[16];  // B^-16k, k < 16
    u64 ibc0;      // B^-256c for the chunk of the first step
    u64 ib256;     // B^-256
    u64 bl1, bl2;  // B^(l1/4 + 1), B^(l2/4 + 1)
    u64 b2[32];    // B^(2^k)
};

// B^L mod p from the table of squares (strings that end inside the round).
__device__ __forceinline__ u64 kr_pow(u64 L, const RoundW &rw)
{
    u64 r = 1;
    for (u32 k = 0; L; k++, L >>= 1)
        if (L & 1) r = mulmod61(r, rw.b2[k]);
    return r;
}

#define RW_STEPS 16  // 64-byte steps per 1024-byte chunk

typedef int v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void_h;

// sum_d v_d 2^(7d) mod p for the ten digit sums v_d < 2^25 of one lane:
// accumulated as a 128-bit integer (< 2^89), then folded with 2^64 = 8.
__device__ __forceinline__ u64 digits_mod61(const v16i &S)
{
    u64 lo = 0, hi = 0;
#pragma unroll
    for (int d = 0; d < 10; d++) {
        const u64 v = (u64)(u32)S[d];
        const u64 a = d ? v << (7 * d) : v;
        const u64 c = (d && 7 * d > 39) ? v >> (64 - 7 * d) : 0ull;
        const u64 t = lo + a;
        hi += c + (t < lo ? 1ull : 0ull);
        lo = t;
    }
    u64 r = (lo & KR_P) + (lo >> 61) + (hi << 3);
    r = (r & KR_P) + (r >> 61);
    return r >= KR_P ? r - KR_P : r;
}

// 16 bytes (two little-endian words) at any byte offset of LDS, from aligned words.
__device__ __forceinline__ void lds_le16(const u8 *R, u32 a, u64 &lo, u64 &hi)
{
    const u32 *p = (const u32 *)(R + (a & ~3u));
    const u32 r = a & 3u;
    u32 d[5];
#pragma unroll
    for (int k = 0; k < 5; k++) d[k] = p[k];
    u32 q[4];
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = __builtin_amdgcn_alignbyte(d[k + 1], d[k], r);  // (r = 0: d[k])
    lo = (u64)q[0] | ((u64)q[1] << 32);
    hi = (u64)q[2] | ((u64)q[3] << 32);
}

#define HF_ACC 3  // first pass: accumulators of two precomputed rounds each (rounds 2a, 2a + 1)

#define HF_CH 5      // 16-byte chunks per string in the first pass (64 bytes at any alignment)
#define HF_ROW 3072  // LDS bytes per wavefront: three 1 KiB copy rows (32 x 5 chunks)

// The first pass over tiles of 32 strings: their first min(len, W) bytes
// (W = the longest precomputed round, <= 64) are copied into LDS by the
// transfer unit, read into registers, and the next tile's copy is issued
// before the current tile's products.  Accumulator a holds rounds 2a (row set
// 0, lane half 0) and 2a + 1 (row set 1, half 1), with the weights of
// positions past the round's length zero; each lane combines its own digit
// sums into G of its rounds and writes their keys; the last round's G is the
// state later rounds continue from.  (When the deep first pass is chosen it
// does this work and more, and this kernel is not launched.)
__global__ __launch_bounds__(256, 4) void k_hash_first(u32 n, const u8 *bytes, u64 N, const u64 *off, PreLens P,
                                                       u32 bits, BPow bp, FirstW fw, u64 *state, u64 *pre, u64 *fl,
                                                       u32 wstate)
{
    __shared__ v4i wtab[HF_ACC][2][2][64];  // [accumulator][32-byte block][low/high product][lane]
    __shared__ __attribute__((aligned(16))) u8 rows[4 * HF_ROW];
    __shared__ u64 pwa[4][32];  // per wavefront: copy start (16-aligned, relative) of each string
    __shared__ u32 pwn[4][32];  // ... and its chunk count (0: not copied)
    __shared__ u64 s_ib[16], s_l[PRE_SLOTS];
    // kernel-argument arrays are read with constant indices only
    if (threadIdx.x < 16) {
        u64 v = 0;
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (threadIdx.x == (u32)k) v = fw.ib[k];
        s_ib[threadIdx.x] = v;
    }
    if (threadIdx.x < PRE_SLOTS) {
        u64 v = 0;
#pragma unroll
        for (int k = 0; k < PRE_SLOTS; k++)
            if (threadIdx.x == (u32)k) v = (u32)k < P.count ? P.l[k] : 0;
        s_l[threadIdx.x] = v;
    }
    __syncthreads();
    for (u32 e = threadIdx.x; e < HF_ACC * 2 * 2 * 64; e += blockDim.x) {
        const u32 ln = e & 63, hl = (e >> 6) & 1, kb = (e >> 7) & 1, a = e >> 8;
        const u32 rc = ln & 31, kh = ln >> 5;
        const u32 dr = 4 * (rc >> 3) + (rc & 3);  // the row's register (digit) in its set
        const u32 r = 2 * a + ((rc >> 2) & 1);     // the row's round
        const bool ok = r < P.count && (hl ? (dr >= 1 && dr < 10) : dr < 9);
        const u32 d = hl ? dr - 1 : dr;
        const u64 lim = ok ? s_l[r < PRE_SLOTS ? r : 0] : 0;
        u32 wd[4] = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const u32 j = 8 * kb + 4 * kh + q;  // limb: positions 4j .. 4j+3
            const u64 ib = s_ib[j];
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const u32 c = (4 * j + b < lim) ? (u32)((rot61(ib, 8 * b) >> (7 * d)) & 127u) : 0u;
                wd[q] |= c << (8 * b);
            }
        }
        wtab[a][kb][hl][ln] = v4i{(int)wd[0], (int)wd[1], (int)wd[2], (int)wd[3]};
    }
    __syncthreads();
    const u32 lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5, wv = threadIdx.x >> 6;
    u8 *R = rows + wv * HF_ROW;
    const u64 babs = (u64)(uintptr_t)bytes;
    const u32 W = (u32)s_l[P.count - 1];
    const u32 nacc = (P.count + 1) / 2;
    u64 fmn[HF_ACC], fmx[HF_ACC], fsh[HF_ACC];
#pragma unroll
    for (int a = 0; a < HF_ACC; a++) {
        fmn[a] = ~0ull;
        fmx[a] = 0;
        fsh[a] = 0;
    }
    const u32 ntiles = (n + 31) / 32;
    const u32 wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwaves = (gridDim.x * blockDim.x) >> 6;
    // copy [0, min(len, W)) of this lane's string into the rows
    auto issue_copy = [&](u64 o, u32 m) {
        const u64 A0 = (babs + o) & ~15ull;
        const u32 sh = (u32)((babs + o) & 15);
        const u32 nch = m ? (sh + m + 15) / 16 : 0u;
        const bool edge = nch && (A0 < babs || A0 + 16ull * nch > babs + N);
        if (h == 0) {  // (read back below by the same wavefront: LDS keeps its order)
            pwa[wv][col] = A0 - babs;
            pwn[wv][col] = edge ? 0u : nch;
        }
        constexpr int T = (32 * HF_CH + 63) / 64;
        u64 ad[T];
        bool ok[T];
#pragma unroll
        for (int t = 0; t < T; t++) {  // every address first: the copies then issue back to back
            u32 slot = 64 * t + lane;
            asm volatile("" : "+v"(slot));  // recomputed per tile rather than held in registers
            const u32 sx = slot / HF_CH, c = slot % HF_CH;
            ad[t] = pwa[wv][sx & 31] + 16u * c;
            ok[t] = sx < 32 && c < pwn[wv][sx & 31];
        }
#pragma unroll
        for (int t = 0; t < T; t++)
            if (ok[t]) __builtin_amdgcn_global_load_lds((const void *)(bytes + ad[t]), (lds_void_h *)(R + 1024 * t), 16, 0, 0);
    };
    auto str_of = [&](u32 tile, u64 &o, u32 &len) {  // offsets of this lane's string of `tile`
        const u32 i = tile * 32 + col;
        const u32 ic = i < n ? i : n - 1;  // loads without a branch; len 0 past the end
        o = off[ic];
        const u64 e = off[ic + 1];
        len = i < n ? (u32)(e - o) : 0u;
    };
    if (wave < ntiles) {
        u32 tile = wave;
        u64 o_c, o_n = 0;
        u32 len_c, len_n = 0;
        str_of(tile, o_c, len_c);
        bool more = tile + nwaves < ntiles;
        if (more) str_of(tile + nwaves, o_n, len_n);
        issue_copy(o_c, len_c < W ? len_c : W);
        for (;;) {  // tiles; uniform over the wavefront
            const u32 m = len_c < W ? len_c : W;
            u64 lo[2], hi[2];
            // vmcnt(0): this tile's copy has landed in the rows (the compiler
            // waits only for loads into registers)
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __asm__ volatile("" ::: "memory");  // (no row read moves above the wait)
            {
                const u32 sh = (u32)((babs + o_c) & 15);
                const u32 nch = m ? (sh + m + 15) / 16 : 0u;
                const u64 A0 = (babs + o_c) & ~15ull;
                const bool edge = nch && (A0 < babs || A0 + 16ull * nch > babs + N);
#pragma unroll
                for (int kb = 0; kb < 2; kb++) {
                    const u32 rel = 32 * kb + 16 * h;
                    const u32 take = m > rel ? ((m - rel) < 16 ? m - rel : 16u) : 0u;
                    lo[kb] = hi[kb] = 0;
                    if (take) {
                        if (!edge) lds_le16(R, HF_CH * 16 * col + sh + rel, lo[kb], hi[kb]);
                        else load16_le(bytes, N, o_c + rel, take, lo[kb], hi[kb]);
                        if (take < 8) {
                            lo[kb] &= (1ull << (8 * take)) - 1ull;
                            hi[kb] = 0;
                        } else if (take < 16) {
                            hi[kb] &= take == 8 ? 0ull : ((1ull << (8 * (take - 8))) - 1ull);
                        }
                    }
                }
            }
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the rows are read before the next copy
            const u32 next = tile + nwaves;
            u64 o_nn = 0;
            u32 len_nn = 0;
            if (more) {
                issue_copy(o_n, len_n < W ? len_n : W);
                if (next + nwaves < ntiles) str_of(next + nwaves, o_nn, len_nn);
            }
            // the tile's products: two per accumulator and block
            v16i S[HF_ACC];
#pragma unroll
            for (int a = 0; a < HF_ACC; a++) S[a] = v16i{};
#pragma unroll
            for (int kb = 0; kb < 2; kb++) {
                const u64 l7 = 0x7F7F7F7F7F7F7F7Full, h1 = 0x0101010101010101ull;
                const u64 lo7 = lo[kb] & l7, hi7 = hi[kb] & l7, loh = (lo[kb] >> 7) & h1, hih = (hi[kb] >> 7) & h1;
                const v4i xl = v4i{(int)(u32)lo7, (int)(u32)(lo7 >> 32), (int)(u32)hi7, (int)(u32)(hi7 >> 32)};
                const v4i xh = v4i{(int)(u32)loh, (int)(u32)(loh >> 32), (int)(u32)hih, (int)(u32)(hih >> 32)};
#pragma unroll
                for (int a = 0; a < HF_ACC; a++) {
                    if ((u32)a >= nacc) break;  // uniform
                    S[a] = __builtin_amdgcn_mfma_i32_32x32x32_i8(wtab[a][kb][0][lane], xl, S[a], 0, 0, 0);
                    S[a] = __builtin_amdgcn_mfma_i32_32x32x32_i8(wtab[a][kb][1][lane], xh, S[a], 0, 0, 0);
                }
            }
            const u32 i = tile * 32 + col;
#pragma unroll
            for (int a = 0; a < HF_ACC; a++) {
                const u32 r = 2 * a + h;
                if ((u32)a >= nacc) break;  // uniform
                if (i < n && r < P.count) {
                    const u64 G = digits_mod61(S[a]);
                    const u32 lr = (u32)s_l[r];
                    const u32 mr = len_c < lr ? len_c : lr;
                    const u64 key = kr_key(G, bp.p[(mr + 3) / 4 + 1], mr, bits);
                    pre[(u64)r * n + i] = key;
                    if (wstate && r == P.count - 1) state[i] = G;  // later rounds continue from G
                    fmn[a] = key < fmn[a] ? key : fmn[a];
                    fmx[a] = key > fmx[a] ? key : fmx[a];
                    if (len_c <= lr) fsh[a] = 1;
                }
            }
            if (!more) break;
            tile = next;
            o_c = o_n;
            len_c = len_n;
            o_n = o_nn;
            len_n = len_nn;
            more = tile + nwaves < ntiles;
        }
    }
#pragma unroll
    for (int a = 0; a < HF_ACC; a++) {
        flags_reduce32(fmn[a], fmx[a], fsh[a]);
        const u32 r = 2 * a + h;
        if (col == 0 && r < P.count) flags_commit(fl + 3 * r, fmn[a], fmx[a], fsh[a]);
    }
}


// Arguments of a hashing pass over a list of strings (the first pass: all strings).
struct PassArgs {
    const u32 *act;    // active list (NULL: strings 0..n-1 in order)
    const u32 *cnt;    // its length (device word); the first pass uses n
    u32 n;             // number of strings (first pass)
    const u8 *bytes;
    u64 N;
    const u64 *off;
    u64 lprev, l1, l2; // continue G from lprev; keys at l1 (and l2 when nonzero)
    u32 bits;
    u64 *state;        // G by string index (in: at lprev; out: at the last round)
    u64 *keys1, *keys2;  // round keys by list position
    u64 *rf;           // flags of rounds l1 (rf[0..2]) and l2 (rf[3..5])
    const v4i *wt;     // deep first pass: the weight tables (round, then first-pass), made by k_hash_weights
    u64 *pre;          // first pass: keys of precomputed round r at pre[r n + i]
    u64 *fl;           // first pass: flags of precomputed round r at fl[3r ..]
};

struct FirstArgs {
    PreLens P;  // rounds up to 64 bytes
    BPow bp;
    FirstW fw;
    // Sort seed (deep pass; null: none): per string, its first mismatch with
    // the first string of its set and its 8 bytes there (see
    // ss_dist_prefix_first_seed).  set_off null: one set.
    u64 *seed_word;
    uint2 *seed_pos;
    const u64 *set_off;
    u32 nsets;
    // lazy: the rounds of at most 64 bytes are not hashed; instead cert gets
    // a lower bound on every string's LCP with string 0 (over at most 256
    // bytes) and minlen the shortest length, from which the caller tells
    // whether those rounds can finish anything (if so it hashes them later)
    u32 lazy;
    u64 *cert, *minlen;
};

#define SEED_MAX_SETS 16  // sets whose first strings the pass keeps in LDS (more: no seed)

#define SEED_OPEN 0xFFFFFFFFu  // seed_pos[i].y of a string not resolved inside the pass

#define WT_ROUND (RW_STEPS * 2 * 2 * 9)  // round weights: [step of the chunk][32-byte block][16-byte half][digit]
#define WT_FIRST (HF_ACC * 2 * 2 * 64)   // first-pass weights: [accumulator][32-byte block][low/high product][lane]

// Round-weight entry e: the four limbs' 7-bit digit d of the 16 positions of
// one step's 32-byte block half, as i8 operands.
__device__ __forceinline__ v4i wtab_entry(u32 e, const RoundW &rw)
{
    const u32 d = e % 9, kh = (e / 9) & 1, kb = (e / 18) & 1, st = e / 36;
    u32 wd[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 4; q++) {  // the four limbs of the 16 positions
        const u32 j = 16 * st + 8 * kb + 4 * kh + q;
        const u64 ib = mulmod61(rw.iblo[j & 15], rw.ibhi[j >> 4]);
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const u32 c = (u32)((rot61(ib, 8 * b) >> (7 * d)) & 127u);
            wd[q] |= c << (8 * b);
        }
    }
    return v4i{(int)wd[0], (int)wd[1], (int)wd[2], (int)wd[3]};
}

// First-pass weight entry e (lane ln of accumulator a): the row's round keeps
// the weights of positions below its length l[r], the rest are zero.
__device__ __forceinline__ v4i wfirst_entry(u32 e, const u64 *ibs, const u64 *l, u32 c0)
{
    const u32 ln = e & 63, hl = (e >> 6) & 1, kb = (e >> 7) & 1, a = e >> 8;
    const u32 rc = ln & 31, kh = ln >> 5;
    const u32 dr = 4 * (rc >> 3) + (rc & 3);  // the row's register (digit) in its set
    const u32 r = 2 * a + ((rc >> 2) & 1);     // the row's round
    const bool ok = r < c0 && (hl ? (dr >= 1 && dr < 10) : dr < 9);
    const u32 d = hl ? dr - 1 : dr;
    const u64 lim = ok ? l[r < PRE_SLOTS ? r : 0] : 0;
    u32 wd[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const u32 j = 8 * kb + 4 * kh + q;  // limb: positions 4j .. 4j+3
        const u64 ib = ibs[j];
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const u32 c = (4 * j + b < lim) ? (u32)((rot61(ib, 8 * b) >> (7 * d)) & 127u) : 0u;
            wd[q] |= c << (8 * b);
        }
    }
    return v4i{(int)wd[0], (int)wd[1], (int)wd[2], (int)wd[3]};
}

// The deep first pass's weight tables (round weights, then first-pass
// weights), once per call: wt[WT_ROUND + WT_FIRST].
__global__ __launch_bounds__(256) void k_hash_weights(RoundW rw, FirstArgs F, v4i *wt)
{
    __shared__ u64 s_ib[16], s_l[PRE_SLOTS];
    const u32 c0 = F.P.count;
    // kernel-argument arrays are read with constant indices only
    if (threadIdx.x < 16) {
        u64 v = 0;
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (threadIdx.x == (u32)k) v = F.fw.ib[k];
        s_ib[threadIdx.x] = v;
    }
    if (threadIdx.x < PRE_SLOTS) {
        u64 v = 0;
#pragma unroll
        for (int k = 0; k < PRE_SLOTS; k++)
            if (threadIdx.x == (u32)k) v = (u32)k < c0 ? F.P.l[k] : 0;
        s_l[threadIdx.x] = v;
    }
    __syncthreads();
    const u32 e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < WT_ROUND) wt[e] = wtab_entry(e, rw);
    else if (e < WT_ROUND + WT_FIRST) wt[e] = wfirst_entry(e - WT_ROUND, s_ib, s_l, c0);
}

// One pass = PS steps of a tile's 32 strings.  Before its products are
// taken, every string's bytes of the pass are copied into the wavefront's LDS
// rows by the transfer unit (chunk c of string s at 16 (CH s + c), from
// the string's 16-aligned pass start), so that each copy instruction reads
// long runs of one string; the lanes then read their MFMA operands from LDS.
// The copy of the next pass is issued before the current pass's products.
//
// FIRST: the deep first pass over all strings (the plain first pass is the
// standalone k_hash_first).  Its rounds up to 64 bytes come from the first
// step: accumulator a holds rounds 2a (row set 0, lane half 0) and 2a + 1
// (set 1, half 1) with the weights of positions past each round's length
// zero, and each lane writes the keys of its rounds.  It continues the same
// read to l2 = 256 and precomputes rounds l1 = 128 and l2 with the round
// machinery, so data whose strings mostly share a long prefix are read once
// instead of in two passes.  The host reads the probe's count back and
// launches one of the two first-pass kernels.
//
// LAZY (deep first pass only): the rounds up to 64 bytes are left out -- the
// pass compares every string with its set's first string instead, and
// certifies how long a prefix they all share (the rounds call hashes those
// rounds afterwards only if that does not prove them unable to finish a
// string).  Without the first step's products and their weight table the
// kernel needs fewer registers and less LDS, and more workgroups fit on a
// compute unit.
//
// NW wavefronts per workgroup (they share the weight tables), PS 64-byte
// steps per pass: CH 16-byte chunks per string cover a pass at any alignment.
template <bool FIRST, bool LAZY = false, int NW = 4, int PS = 2>
__device__ __forceinline__ void hash_pass(const PassArgs &A, const RoundW &rw, const FirstArgs *Fp)
{
    static_assert(FIRST || !LAZY, "only the deep first pass leaves rounds out");
    constexpr int CH = 4 * PS + 1;
    constexpr int ROW = 512 * CH + 64;  // LDS bytes of a wavefront's rows (32 strings; a read may run 4 past)
    // round weights: [step of the chunk][32-byte block][16-byte half][digit]
    __shared__ v4i wtab[WT_ROUND + 1];  // (and a zero entry, for rows left out)
    // first-pass weights: [accumulator][32-byte block][low/high product][lane]
    __shared__ v4i wfirst[(FIRST && !LAZY) ? WT_FIRST : 1];
    __shared__ __attribute__((aligned(16))) u8 rows[NW * ROW];
    __shared__ u64 pwa[NW][32];  // per wavefront: pass start (16-aligned, relative) of each string
    __shared__ u32 pwn[NW][32];  // ... and its chunk count (0: not copied)
    __shared__ u64 s_l[PRE_SLOTS];
    if (threadIdx.x == 0) wtab[WT_ROUND] = v4i{0, 0, 0, 0};
    if (FIRST) {  // the same tables for every workgroup: made once per call
        for (u32 e = threadIdx.x; e < WT_ROUND; e += blockDim.x) wtab[e] = A.wt[e];
        if (!LAZY)
            for (u32 e = threadIdx.x; e < WT_FIRST; e += blockDim.x) wfirst[e] = A.wt[WT_ROUND + e];
    } else {
        for (u32 e = threadIdx.x; e < WT_ROUND; e += blockDim.x) wtab[e] = wtab_entry(e, rw);
    }
    u32 c0 = 0;  // precomputed rounds up to 64 bytes (first pass)
    // Sort seed: the set bounds and, per set, the first 4 * PRE_MAX bytes
    // (zero past its end) and the length of its reference string -- the
    // set's first string -- all in LDS.  (The strings of a tile across sets,
    // at most 32 per set boundary, are left for the sort to compare from the
    // start.)
    __shared__ u64 s_set[FIRST ? SEED_MAX_SETS + 1 : 1];
    __shared__ __attribute__((aligned(16))) u64 s_ref[FIRST ? SEED_MAX_SETS : 1][FIRST ? PRE_MAX / 2 : 1];
    __shared__ u32 s_refl[FIRST ? SEED_MAX_SETS : 1];
    __shared__ u64 s_mw[FIRST ? NW : 1][32];  // per wavefront and string: the 8 bytes at its record
    const bool seeding = FIRST && Fp->seed_pos != nullptr;  // uniform: seed records are written
    constexpr bool lazy = LAZY;                              // the rounds up to 64 bytes are left out
    const bool comparing = seeding || lazy;                  // the strings are compared with their references
    const u32 nsets = (FIRST && comparing && Fp->set_off) ? Fp->nsets : 1u;  // (<= SEED_MAX_SETS)
    if (FIRST) {
        const FirstArgs &F = *Fp;
        c0 = F.P.count;
        if (comparing) {
            for (u32 e = threadIdx.x; e <= nsets; e += blockDim.x)
                s_set[e] = F.set_off ? F.set_off[e] : (e ? (u64)A.n : 0ull);
            for (u32 e = threadIdx.x; e < nsets * (PRE_MAX / 2); e += blockDim.x) {
                const u32 sx = e / (PRE_MAX / 2), k = 8 * (e % (PRE_MAX / 2));
                u64 f = F.set_off ? F.set_off[sx] : 0ull;
                f = f < A.n ? f : A.n - 1;  // (bounds that are not well placed stay inside the arrays)
                const u64 fo = A.off[f], fl64 = A.off[f + 1] - fo;
                const u32 fl = fl64 < 0xFFFFFFFFull ? (u32)fl64 : 0xFFFFFFFFu;
                s_ref[sx][k / 8] = k < fl ? load_le(A.bytes, A.N, fo + k, (fl - k) < 8 ? fl - k : 8u) : 0ull;
                if (k == 0) s_refl[sx] = fl;
            }
        }
        // kernel-argument arrays are read with constant indices only
        if (threadIdx.x < PRE_SLOTS) {
            u64 v = 0;
#pragma unroll
            for (int k = 0; k < PRE_SLOTS; k++)
                if (threadIdx.x == (u32)k) v = (u32)k < c0 ? F.P.l[k] : 0;
            s_l[threadIdx.x] = v;
        }
    }
    __syncthreads();
    const u32 lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5, wv = threadIdx.x >> 6;
    u8 *R = rows + wv * ROW;
    const u64 babs = (u64)(uintptr_t)A.bytes;
    const u8 *bytes = A.bytes;
    const u64 N = A.N;
    const u64 *off = A.off;
    // this lane's weight row: register dr of row set 0 (full weights) or set 1
    // (weights below l1); digit dr in the low-bit product, dr - 1 in the high-bit one
    const u32 dr = 4 * (col >> 3) + (col & 3);
    const bool rowl1 = (col & 4) != 0;
    const bool rowlo = dr < 9, rowhi = dr >= 1 && dr < 10;
    // positions inside a string fit in 32 bits
    const bool two = A.l2 != 0;
    const u32 L1 = (u32)A.l1, LP = FIRST ? 0u : (u32)A.lprev;
    const u32 lend = two ? (u32)A.l2 : L1;
    const u32 lmine = (two && h) ? L1 : lend;  // the round this lane finishes
    // B^(lmine/4 + 1), selected bitwise (a select of the two loads becomes an
    // indexed stack array)
    const u64 selm = 0ull - (u64)(lmine == L1);
    const u64 blmine = (rw.bl1 & selm) | (rw.bl2 & ~selm);
    // (the same for the output of half 0's keys)
    const u64 sel2 = 0ull - (u64)two;
    u64 *const keys0 = (u64 *)(((uintptr_t)A.keys2 & sel2) | ((uintptr_t)A.keys1 & ~sel2));
    const u32 nacc = (c0 + 1) / 2;
    // Flags of this lane's keys, per slot (the first pass's accumulators 0..2,
    // then the round machinery): the first key seen, and bits 3s (a key was
    // seen), 3s + 1 (a later key differed from it), 3s + 2 (a string was no
    // longer than the round) -- all a round's keys are equal iff no lane saw
    // two different ones and every lane's first key is the same.
    u64 fk[HF_ACC + 1];
#pragma unroll
    for (int a = 0; a <= HF_ACC; a++) fk[a] = 0;
    u32 fb = 0;
    auto note = [&](int slot, u64 key, bool shrt) {
        const u32 hv = 1u << (3 * slot);
        const bool seen = (fb & hv) != 0;
        fb |= hv | ((seen && key != fk[slot]) ? hv << 1 : 0u) | (shrt ? hv << 2 : 0u);
        fk[slot] = seen ? fk[slot] : key;
    };
    // The flags of one slot as a minimum, maximum and short flag.  In the
    // deep first pass each wavefront half's go to LDS and the workgroup's are
    // committed once per lane half (the few global words take 4x fewer
    // atomics); round passes commit per wavefront half.
    __shared__ u64 s_fmn[FIRST ? HF_ACC + 1 : 1][NW][2], s_fmx[FIRST ? HF_ACC + 1 : 1][NW][2];
    __shared__ u32 s_fsh[FIRST ? HF_ACC + 1 : 1][NW][2];
    auto stage = [&](int slot) {
        const u32 b = fb >> (3 * slot);
        u64 mn = (b & 1) ? ((b & 2) ? 0ull : fk[slot]) : ~0ull;
        u64 mx = (b & 1) ? ((b & 2) ? ~0ull : fk[slot]) : 0ull;
        u64 sh = (b >> 2) & 1;
        flags_reduce32(mn, mx, sh);
        if (col == 0) {
            s_fmn[slot][wv][h] = mn;
            s_fmx[slot][wv][h] = mx;
            s_fsh[slot][wv][h] = (u32)sh;
        }
    };
    auto commit = [&](int slot, u64 *f, bool doit) {  // (after a barrier)
        if (wv == 0 && col == 0 && doit) {
            u64 mn = ~0ull, mx = 0, sh = 0;
#pragma unroll
            for (int w = 0; w < NW; w++) {
                const u64 a = s_fmn[slot][w][h], b = s_fmx[slot][w][h];
                mn = a < mn ? a : mn;
                mx = b > mx ? b : mx;
                sh |= s_fsh[slot][w][h];
            }
            flags_commit(f, mn, mx, sh);
        }
    };
    const u32 Acnt = FIRST ? A.n : *A.cnt;
    const u32 ntiles = (Acnt + 31) / 32;
    const u32 wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwaves = (gridDim.x * blockDim.x) >> 6;
    const u32 x0 = LP & ~63u;
    // Indices past the list are clamped to its last entry so that the loads
    // need no branch.
    auto entry = [&](u32 tile) -> u32 {
        const u32 jj = tile * 32 + col;
        const u32 jc = jj < Acnt ? jj : Acnt - 1;
        return A.act ? A.act[jc] : jc;
    };
    auto tile_xmax = [&](u32 m) -> u32 {
#pragma unroll
        for (int s2 = 1; s2 < 32; s2 <<= 1) {
            const u32 t = __shfl_xor(m, s2);
            m = t > m ? t : m;
        }
        return m;
    };
    // copy pass [xp, xp + 128) of this lane's string (string end m) into the rows
    auto issue_copy = [&](u64 o, u32 m, u32 xp) {
        const u64 A0 = (babs + o + xp) & ~15ull;
        const u32 sh = (u32)((babs + o + xp) & 15);
        const u32 need = m > xp ? ((m - xp < 64 * PS ? m : xp + 64 * PS) - xp) : 0u;
        const u32 nch = need ? (sh + need + 15) / 16 : 0u;
        const bool edge = nch && (A0 < babs || A0 + 16ull * nch > babs + N);
        if (h == 0) {  // (read back below by the same wavefront: LDS keeps its order)
            pwa[wv][col] = A0 - babs;
            pwn[wv][col] = edge ? 0u : nch;
        }
        constexpr int T = (32 * CH + 63) / 64;
        u64 ad[T];
        bool ok[T];
#pragma unroll
        for (int t = 0; t < T; t++) {  // every address first: the copies then issue back to back
            u32 slot = 64 * t + lane;
            asm volatile("" : "+v"(slot));  // recomputed per pass rather than held in registers
            const u32 sx = slot / CH, c = slot % CH;
            ad[t] = pwa[wv][sx & 31] + 16u * c;
            ok[t] = sx < 32 && c < pwn[wv][sx & 31];
        }
#pragma unroll
        for (int t = 0; t < T; t++)
            if (ok[t]) __builtin_amdgcn_global_load_lds((const void *)(bytes + ad[t]), (lds_void_h *)(R + 1024 * t), 16, 0, 0);
    };
    if (wave < ntiles) {
        // current tile: entry, offsets, state; the next tile's entry
        u32 tile = wave;
        u32 i_c = entry(tile);
        bool valid = tile * 32 + col < Acnt;
        u64 o_c = off[i_c];
        u32 len = valid ? (u32)(off[i_c + 1] - o_c) : 0u;
        u64 G = (valid && LP) ? A.state[i_c] : 0ull;
        u32 i_n = entry(tile + nwaves < ntiles ? tile + nwaves : tile);
        u64 o_n = 0, G_n = 0;
        u32 len_n = 0;
        bool more = tile + nwaves < ntiles;
        if (more) {
            o_n = off[i_n];
            len_n = (u32)(off[i_n + 1] - o_n);
            if (LP) G_n = A.state[i_n];
        }
        u32 i_nn = entry(tile + 2 * nwaves < ntiles ? tile + 2 * nwaves : tile);
        u32 m = len < lend ? len : lend;
        u32 xmax = tile_xmax(m);
        u64 ibc = rw.ibc0;
        v16i S = {};
        u32 xp = x0;
        u32 smis = 0xFFFFFFFFu;  // sort seed: first byte of this lane's pieces unlike the reference's
        u32 cmin = 0xFFFFFFFFu, lmin = 0xFFFFFFFFu;  // lazy: this lane's certified LCP, shortest length
        bool mwgot = false;      // ... the string's 8 bytes at its record are in s_mw
        u32 runi = 1;            // the tile's strings share one set (uniform)
        u32 rsel = 0;            // ... which one (uniform)
        // the set of the tile's strings
        auto seed_ref = [&](u32 t) {
            const u32 jc = t * 32 + col < Acnt ? t * 32 + col : Acnt - 1;
            u32 slo = 0, shi = nsets;  // the last set starting at or before jc
            while (shi - slo > 1) {
                const u32 mid = (slo + shi) >> 1;
                if (s_set[mid] <= jc) slo = mid;
                else shi = mid;
            }
            runi = __builtin_amdgcn_readfirstlane((u32)(__shfl(slo, 0, 64) == __shfl(slo, 31, 64)));
            rsel = __builtin_amdgcn_readfirstlane(slo);
        };
        if (FIRST && comparing) seed_ref(tile);
        issue_copy(o_c, m, xp);
        for (;;) {  // passes; uniform over the wavefront
            // this pass's operand bytes: [u][kb], 16 each (zero past the string)
            u64 lo[PS][2], hi[PS][2];
            bool top;  // (uniform) some byte of the pass is >= 128
            // vmcnt(0): this pass's copy has landed in the rows (the compiler
            // waits only for loads into registers)
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __asm__ volatile("" ::: "memory");  // (no row read moves above the wait)
            {
                const u32 sh = (u32)((babs + o_c + xp) & 15);
                const u32 need = m > xp ? ((m - xp < 64 * PS ? m : xp + 64 * PS) - xp) : 0u;
                const u32 nch = need ? (sh + need + 15) / 16 : 0u;
                const u64 A0 = (babs + o_c + xp) & ~15ull;
                const bool edge = nch && (A0 < babs || A0 + 16ull * nch > babs + N);
                if (__all(!edge && need == 64 * PS)) {
                    // every lane's pass is whole and in its rows
#pragma unroll
                    for (int u = 0; u < PS; u++)
#pragma unroll
                        for (int kb = 0; kb < 2; kb++)
                            lds_le16(R, CH * 16 * col + sh + 64 * u + 32 * kb + 16 * h, lo[u][kb], hi[u][kb]);
                } else {
#pragma unroll
                    for (int u = 0; u < PS; u++)
#pragma unroll
                        for (int kb = 0; kb < 2; kb++) {
                            const u32 rel = 64 * u + 32 * kb + 16 * h;
                            const u32 take = need > rel ? ((need - rel) < 16 ? need - rel : 16u) : 0u;
                            lo[u][kb] = hi[u][kb] = 0;
                            if (take) {
                                if (!edge) lds_le16(R, CH * 16 * col + sh + rel, lo[u][kb], hi[u][kb]);
                                else load16_le(bytes, N, o_c + xp + rel, take, lo[u][kb], hi[u][kb]);
                                if (take < 8) {
                                    lo[u][kb] &= (1ull << (8 * take)) - 1ull;
                                    hi[u][kb] = 0;
                                } else if (take < 16) {
                                    hi[u][kb] &= take == 8 ? 0ull : ((1ull << (8 * (take - 8))) - 1ull);
                                }
                            }
                        }
                }
                // bytes of 128 or more anywhere in the wavefront's pass: the
                // products then take the low 7 bits and the top bit apart
                {
                    u64 hb = 0;
#pragma unroll
                    for (int u = 0; u < PS; u++)
#pragma unroll
                        for (int kb = 0; kb < 2; kb++) hb |= lo[u][kb] | hi[u][kb];
                    top = __ballot((hb & 0x8080808080808080ull) != 0) != 0;
                }
                if (FIRST && comparing && runi) {
                    // this lane's pieces against the reference's bytes at the same
                    // positions (both zero past their ends; a difference at or
                    // past the shorter end is discarded below): the first
                    // differing word, from the pieces in decreasing position
                    u64 fw = 0;
                    u32 fp = 0;
#pragma unroll
                    for (int u = PS - 1; u >= 0; u--)
#pragma unroll
                        for (int kb = 1; kb >= 0; kb--) {
                            const u32 pos = xp + 64 * u + 32 * kb + 16 * h;
                            if (pos < 4 * PRE_MAX) {
                                typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
                                const u64x2 rv = *(const u64x2 *)&s_ref[rsel][pos / 8];
                                const u64 d0 = lo[u][kb] ^ rv.x, d1 = hi[u][kb] ^ rv.y;
                                if (d1) { fw = d1; fp = pos + 8; }
                                if (d0) { fw = d0; fp = pos; }
                            }
                        }
                    if (fw) {
                        const u32 mp = fp + (u32)(__builtin_ctzll(fw) >> 3);
                        smis = mp < smis ? mp : smis;
                    }
                    // The string's record position so far (its first mismatch,
                    // or the shorter end).  Passes go up in position, so once it
                    // lies in this pass it is final: its 8 bytes are taken from
                    // this pass's rows while they are still there (from global
                    // memory at the tile's end when they reach past the copy).
                    const u32 y = __shfl_xor(smis, 32, 64);
                    const u32 sm = y < smis ? y : smis;
                    const u32 rfl = s_refl[rsel];
                    const u32 E = len < rfl ? len : rfl;
                    const u32 rc = sm < E ? sm : E;
                    if (seeding && !h && rc >= xp && rc < xp + 64 * PS) {
                        const u32 tk = len - rc < 8 ? len - rc : 8u;
                        if (tk == 0) {
                            s_mw[wv][col] = 0;
                            mwgot = true;
                        } else if (!edge && nch && rc + tk <= xp + 16 * nch - sh) {
                            u64 w0, w1;
                            lds_le16(R, CH * 16 * col + sh + (rc - xp), w0, w1);
                            s_mw[wv][col] = __builtin_bswap64(tk < 8 ? (w0 & ((1ull << (8 * tk)) - 1ull)) : w0);
                            mwgot = true;
                        }
                    }
                }
            }
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the rows are read before the next copy
            // the next pass: the rest of this tile, or the next tile's first
            const bool tile_end = xp + 64 * PS >= xmax;
            u32 m_n = 0, xmax_n = 0;
            bool valid_n = false;
            if (!tile_end) {
                issue_copy(o_c, m, xp + 64 * PS);
            } else if (more) {
                valid_n = (tile + nwaves) * 32 + col < Acnt;
                if (!valid_n) len_n = 0;
                m_n = len_n < lend ? len_n : lend;
                xmax_n = tile_xmax(m_n);
                issue_copy(o_n, m_n, x0);
            }
            // this pass's products
#pragma unroll
            for (int u = 0; u < PS; u++) {
                const u32 x = xp + 64 * u;
                const bool fstep = FIRST && x == 0 && !lazy;  // the first pass's rounds (taken even for empty strings)
                if (x >= xmax && !fstep) break;      // uniform over the wavefront
                const u32 sidx = (x & 1023) >> 6;
                v4i xl[2], xh[2];
#pragma unroll
                for (int kb = 0; kb < 2; kb++) {
                    u64 l0 = lo[u][kb], h0 = hi[u][kb];
                    const u32 a0 = x + 32 * kb + 16 * h;
                    if (a0 < LP) {  // bytes below lprev are in G already
                        const u32 skip = LP - a0 < 16 ? LP - a0 : 16u;
                        if (skip >= 8) {
                            l0 = 0;
                            h0 &= skip == 16 ? 0ull : ~((1ull << (8 * (skip - 8))) - 1ull);
                        } else {
                            l0 &= ~((1ull << (8 * skip)) - 1ull);
                        }
                    }
                    // this lane's weight row for the block's 16 positions (lane half = 16-byte
                    // half); rows of the l1 set are zero from l1 on (a two-round l1 is a
                    // multiple of 64, so no block straddles it; single rounds do not use it)
                    const u32 wb = ((sidx * 2 + kb) * 2 + h) * 9;
                    const bool zero = rowl1 && x + 32 * kb >= L1;
                    const v4i wl = wtab[(rowlo && !zero) ? wb + dr : (u32)WT_ROUND];
                    if (!top && !fstep) {
                        // every byte < 128: the bytes are their own low 7 bits, no top-bit product
                        xl[kb] = v4i{(int)(u32)l0, (int)(u32)(l0 >> 32), (int)(u32)h0, (int)(u32)(h0 >> 32)};
                        S = __builtin_amdgcn_mfma_i32_32x32x32_i8(wl, xl[kb], S, 0, 0, 0);
                    } else {
                        const u64 l7 = 0x7F7F7F7F7F7F7F7Full, h1 = 0x0101010101010101ull;
                        const u64 lo7 = l0 & l7, hi7 = h0 & l7, loh = (l0 >> 7) & h1, hih = (h0 >> 7) & h1;
                        xl[kb] = v4i{(int)(u32)lo7, (int)(u32)(lo7 >> 32), (int)(u32)hi7, (int)(u32)(hi7 >> 32)};
                        xh[kb] = v4i{(int)(u32)loh, (int)(u32)(loh >> 32), (int)(u32)hih, (int)(u32)(hih >> 32)};
                        const v4i wh = wtab[(rowhi && !zero) ? wb + dr - 1 : (u32)WT_ROUND];
                        S = __builtin_amdgcn_mfma_i32_32x32x32_i8(wl, xl[kb], S, 0, 0, 0);
                        S = __builtin_amdgcn_mfma_i32_32x32x32_i8(wh, xh[kb], S, 0, 0, 0);
                    }
                }
                if (fstep) {
                    // the precomputed rounds, one accumulator at a time: keys of this
                    // lane's rounds 2a + h
                    const u32 i = tile * 32 + col;
#pragma unroll
                    for (int a = 0; a < HF_ACC; a++) {
                        if ((u32)a >= nacc) break;  // uniform
                        v16i S1 = {};
#pragma unroll
                        for (int kb = 0; kb < 2; kb++) {
                            S1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(wfirst[((a * 2 + kb) * 2 + 0) * 64 + lane], xl[kb], S1, 0, 0, 0);
                            S1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(wfirst[((a * 2 + kb) * 2 + 1) * 64 + lane], xh[kb], S1, 0, 0, 0);
                        }
                        const u32 r = 2 * a + h;
                        if (i < Acnt && r < c0) {
                            const u64 Gr = digits_mod61(S1);
                            const u32 lr = (u32)s_l[r];
                            const u32 mr = len < lr ? len : lr;
                            const u64 key = kr_key(Gr, Fp->bp.p[(mr + 3) / 4 + 1], mr, A.bits);
                            A.pre[(u64)r * Acnt + i] = key;
                            note(a, key, len <= lr);
                        }
                    }
                }
                const u32 xn = x + 64;
                if ((xn & 1023) == 0 || xn >= xmax) {
                    // (half 1: the sum below l1; its rows are zero from l1 on)
                    G = addmod61(G, mulmod61(digits_mod61(S), ibc));
                    S = v16i{};
                    if ((xn & 1023) == 0) ibc = mulmod61(ibc, rw.ib256);
                }
            }
            if (!tile_end) {
                xp += 64 * PS;
                continue;
            }
            // sort seed: the string's first mismatch with its reference over
            // both lane halves; the load of its 8 bytes there is issued here
            // and stored after the keys below
            u64 mw = 0;
            uint2 sp = make_uint2(0u, SEED_OPEN);
            if (FIRST && comparing) {
                const u32 y = __shfl_xor(smis, 32, 64);
                smis = y < smis ? y : smis;
                const u32 rfl = s_refl[rsel];
                const u32 E = len < rfl ? len : rfl;  // compared up to the shorter end
                const u32 r = smis < E ? smis : E;
                if (lazy && valid) {
                    // LCP with the reference (capped at 256 or the shorter end; a
                    // tile across sets certifies nothing), and the length
                    const u32 c = runi ? r : 0u;
                    cmin = c < cmin ? c : cmin;
                    lmin = len < lmin ? len : lmin;
                }
                // equal over [0, lend): the sort goes on from lend (across sets: from 0)
                sp = make_uint2(runi ? lend : 0u, SEED_OPEN);
                if (seeding && valid && !h && runi && (r < lend || E <= lend)) {
                    const u32 tk = len - r < 8 ? len - r : 8u;
                    mw = mwgot ? s_mw[wv][col] : (tk ? load_be(bytes, N, o_c + r, tk) : 0ull);
                    sp = make_uint2(r, tk);
                }
                smis = 0xFFFFFFFFu;
                mwgot = false;
            }
            // the tile's keys of the round machinery
            if (valid && (!h || two)) {
                const u32 j = tile * 32 + col;
                const u32 mm = len < lmine ? len : lmine;
                const u64 key = kr_key(G, mm == lmine ? blmine : kr_pow((mm + 3) / 4 + 1, rw), mm, A.bits);
                if (FIRST) {  // precomputed rounds c0 (l1) and c0 + 1 (l2), by string index
                    A.pre[(u64)(c0 + (h ? 0u : 1u)) * Acnt + j] = key;
                    if (!h) A.state[j] = G;
                } else if (h) {
                    A.keys1[j] = key;
                } else {
                    A.state[i_c] = G;
                    keys0[j] = key;
                }
                note(HF_ACC, key, len <= lmine);
            }
            if (FIRST && seeding && valid && !h) {
                const u32 j = tile * 32 + col;
                Fp->seed_word[j] = mw;
                Fp->seed_pos[j] = sp;
            }
            if (!more) break;
            // advance: the next tile becomes current (its first pass is in flight)
            tile += nwaves;
            i_c = i_n;
            o_c = o_n;
            valid = valid_n;
            len = len_n;
            m = m_n;
            xmax = xmax_n;
            G = valid ? G_n : 0;
            ibc = rw.ibc0;
            xp = x0;
            more = tile + nwaves < ntiles;
            i_n = i_nn;
            if (more) {
                o_n = off[i_n];
                len_n = (u32)(off[i_n + 1] - o_n);
                if (LP) G_n = A.state[i_n];
            }
            i_nn = entry(tile + 2 * nwaves < ntiles ? tile + 2 * nwaves : tile);
            if (FIRST && comparing) seed_ref(tile);
        }
        if (FIRST && lazy) {
            // one atomic per wavefront for the certificate and the length
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const u32 y = __shfl_xor(cmin, o, 64), z = __shfl_xor(lmin, o, 64);
                cmin = y < cmin ? y : cmin;
                lmin = z < lmin ? z : lmin;
            }
            if (lane == 0) {
                atomicMin((unsigned long long *)Fp->cert, (unsigned long long)cmin);
                atomicMin((unsigned long long *)Fp->minlen, (unsigned long long)lmin);
            }
        }
    }
    if (FIRST && lazy && blockIdx.x == 0 && threadIdx.x < nsets) {
        // every reference's LCP with string 0 over the staged bytes
        const u32 sx = threadIdx.x;
        const u32 E = s_refl[sx] < s_refl[0] ? s_refl[sx] : s_refl[0];
        u32 c = 4 * PRE_MAX;
        for (u32 q = 0; q < PRE_MAX / 2; q++) {
            const u64 d = s_ref[sx][q] ^ s_ref[0][q];
            if (d) {
                c = 8 * q + (u32)(__builtin_ctzll(d) >> 3);
                break;
            }
        }
        c = c < E ? c : E;
        atomicMin((unsigned long long *)Fp->cert, (unsigned long long)c);
    }
    if constexpr (FIRST) {
        stage(HF_ACC);
        if (!LAZY) {
#pragma unroll
            for (int a = 0; a < HF_ACC; a++) stage(a);
        }
        __syncthreads();
        // rounds l1 (lane half 1) and l2 (half 0) as precomputed rounds c0, c0 + 1
        commit(HF_ACC, A.fl + 3 * (c0 + (h ? 0u : 1u)), true);
        if (!LAZY) {  // (lazy: nothing was hashed for them)
#pragma unroll
            for (int a = 0; a < HF_ACC; a++) {
                const u32 r = 2 * a + h;
                commit(a, A.fl + 3 * r, r < c0);
            }
        }
    } else {  // A.rf[0..2] round l1, A.rf[3..5] round l2, per wavefront half
        const u32 b = fb >> (3 * HF_ACC);
        u64 mn = (b & 1) ? ((b & 2) ? 0ull : fk[HF_ACC]) : ~0ull;
        u64 mx = (b & 1) ? ((b & 2) ? ~0ull : fk[HF_ACC]) : 0ull;
        u64 sh = (b >> 2) & 1;
        flags_reduce32(mn, mx, sh);
        if (col == 0 && (!h || two)) flags_commit(A.rf + ((two && !h) ? 3 : 0), mn, mx, sh);
    }
}

__global__ __launch_bounds__(256, 4) void k_hash_round(PassArgs A, RoundW rw)
{
    hash_pass<false>(A, rw, nullptr);
}

__global__ __launch_bounds__(256, 3) void k_hash_first_deep(PassArgs A, RoundW rw, FirstArgs F)
{
    hash_pass<true>(A, rw, &F);
}

// Three workgroups per CU: at four the pass spills 36 bytes per lane.
__global__ __launch_bounds__(256, 3) void k_hash_first_lazy(PassArgs A, RoundW rw, FirstArgs F)
{
    hash_pass<true, true>(A, rw, &F);
}

// ------------------------------------------------------------ duplicates
//
// The all-ones word marks an empty slot.  The global table's slots hold a
// key's low 32 bits and a list position (< 2^32 - 1, so never all ones); the
// LDS tables of the bucket form hold keys, which are < 2^61 (residues mod
// 2^61-1, possibly masked to fewer bits), with bit 62 marking a key seen twice
// or more.

#define TAB_EMPTY 0xFFFFFFFFFFFFFFFFull
#define TAB_DUP (1ull << 62)

enum { DM_TABLE = 0, DM_ALLDUP = 1, DM_UNIQUE = 2 };

// (64-bit slot arithmetic: tables of 2^32 slots and more, for n > 2^31 keys)
__device__ __forceinline__ u64 tab_slot(u64 key, u32 logT)
{
    return (key * 0x9E3779B97F4A7C15ull) >> (64 - logT);  // Fibonacci hashing
}

// Key of active entry j: by list position (hash rounds) or by input index
// (rounds hashed in the first pass).
__device__ __forceinline__ u64 key_of(const u64 *keys, int kin, u32 i, u32 j) { return keys[kin ? i : j]; }

__global__ void k_store_u32(u32 *p, u32 v) { *p = v; }
__global__ void k_store_u64(u64 *p, u64 v) { *p = v; }

// For one round over the active list: flags[0] = 1 if some key differs from
// the first entry's, flags[1] = 1 if some string has length <= l.  A round
// with neither (and at least two strings) changes nothing.
__global__ __launch_bounds__(256) void k_flags(const u64 *keys, int kin, const u32 *act, const u32 *cnt,
                                               const u64 *off, u64 l, u32 *flags)
{
    const u32 A = *cnt;
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    bool d = false, sh = false;
    if (j < A) {
        const u32 i = act ? act[j] : j;
        const u32 i0 = act ? act[0] : 0u;
        d = key_of(keys, kin, i, j) != key_of(keys, kin, i0, 0);
        sh = off[i + 1] - off[i] <= l;
    }
    const u64 bd = __ballot(d), bs = __ballot(sh);
    if ((threadIdx.x & 63) == 0) {
        if (bd) flags[0] = 1u;
        if (bs) flags[1] = 1u;
    }
}

// Insert every active key into the table (linear probing).  A slot holds the
// low 32 bits of a key and the list position of the entry that brought it
// first; an entry that finds its key there (the low bits equal, and the key
// at that position equal) marks itself and that entry as duplicates in dupf,
// so that the finishing pass reads one byte per entry, in list order, instead
// of probing the table again.  dupf is zero on entry.  The table has at least
// twice as many slots as keys, so every probe sequence ends.
__global__ __launch_bounds__(256) void k_tab_insert(const u64 *keys, int kin, const u32 *act, const u32 *cnt,
                                                    u64 *tab, u32 logT, u8 *dupf)
{
    const u32 A = *cnt;
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A) return;
    const u32 i = act ? act[j] : j;
    const u64 key = key_of(keys, kin, i, j);
    const u64 low = key & 0xFFFFFFFFull;
    const u64 mine = (low << 32) | j;  // (j < 2^32 - 1: never the empty word)
    const u64 mask = (1ull << logT) - 1ull;
    u64 s = tab_slot(key, logT);
    for (u64 probe = 0; probe <= mask; probe++, s = (s + 1) & mask) {
        u64 cur = __hip_atomic_load(&tab[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == TAB_EMPTY) {
            cur = atomicCAS((unsigned long long *)&tab[s], TAB_EMPTY, mine);
            if (cur == TAB_EMPTY) return;  // inserted
        }
        if ((cur >> 32) == low) {
            const u32 jo = (u32)cur;
            if (key_of(keys, kin, act ? act[jo] : jo, jo) == key) {
                dupf[j] = 1;
                dupf[jo] = 1;
                return;
            }
        }
    }
}

// ---- duplicate detection by buckets (App. B finds multiplicities by sorting
// (hash, index) pairs; here the pairs are only partitioned, by the top bits of
// a mixed key, into buckets small enough to count in LDS).  Three launches and
// one scan: each workgroup counts its contiguous chunk of the list per bucket
// (a bucket-major matrix of counts, so that one scan gives every workgroup's
// range in every bucket), writes its (key, list position) pairs there, and one
// workgroup per bucket counts the keys in an LDS table and writes a duplicate
// flag per list position.  The global table remains for very long lists.
#define DD_NT 256
#define DD_MAXLOG 14                 // at most 2^14 buckets (a workgroup's counts in LDS)
#define DD_HM_CAP (1u << 22)         // counts matrix: buckets x workgroups
#define DD_TSLOTS 8192               // LDS table slots of a bucket pass (64 KB)
#define DD_CAP (DD_TSLOTS / 2 - DD_NT)  // new keys a pass takes before it starts over with more passes
#define DD_MIN_ACT (1u << 16)        // shorter lists use the global table (it fits in L2)
#define DD_MAX_ACT (1u << 26)        // ... and so do longer ones

__device__ __forceinline__ u32 dd_bucket(u64 key, u32 logB)
{
    return logB ? (u32)((key * 0x9E3779B97F4A7C15ull) >> (64 - logB)) : 0u;
}
__device__ __forceinline__ u32 dd_sub(u64 key) { return (u32)((key * 0xC2B2AE3D27D4EB4Full) >> 40); }
__device__ __forceinline__ u32 dd_slot(u64 key) { return (u32)((key * 0x165667B19E3779F9ull) >> 51); }  // 13 bits

// Counts of this workgroup's chunk [w C, (w+1) C) of the list per bucket, into
// hm[b G + w] (every entry of the column written).
__global__ __launch_bounds__(DD_NT) void k_dd_count(const u64 *keys, int kin, const u32 *act, const u32 *cnt,
                                                    u32 logB, u32 C, u32 G, u32 *hm)
{
    __shared__ u32 h[1u << DD_MAXLOG];
    const u32 NB = 1u << logB;
    for (u32 b = threadIdx.x; b < NB; b += DD_NT) h[b] = 0;
    __syncthreads();
    const u32 A = *cnt;
    const u32 j0 = blockIdx.x * C, j1 = min(A, j0 + C);
    for (u32 j = j0 + threadIdx.x; j < j1; j += DD_NT) {
        const u32 i = act ? act[j] : j;
        atomicAdd(&h[dd_bucket(key_of(keys, kin, i, j), logB)], 1u);
    }
    __syncthreads();
    for (u32 b = threadIdx.x; b < NB; b += DD_NT) hm[(u64)b * G + blockIdx.x] = h[b];
}

// The same chunk's pairs into their buckets: hm now holds the exclusive scan
// of the counts (bucket-major), i.e. where this workgroup's pairs of each
// bucket start.
__global__ __launch_bounds__(DD_NT) void k_dd_scatter(const u64 *keys, int kin, const u32 *act, const u32 *cnt,
                                                      u32 logB, u32 C, u32 G, const u32 *hm, u64 *pk, u32 *pj)
{
    __shared__ u32 h[1u << DD_MAXLOG];
    const u32 NB = 1u << logB;
    for (u32 b = threadIdx.x; b < NB; b += DD_NT) h[b] = hm[(u64)b * G + blockIdx.x];
    __syncthreads();
    const u32 A = *cnt;
    const u32 j0 = blockIdx.x * C, j1 = min(A, j0 + C);
    for (u32 j = j0 + threadIdx.x; j < j1; j += DD_NT) {
        const u32 i = act ? act[j] : j;
        const u64 key = key_of(keys, kin, i, j);
        const u32 slot = atomicAdd(&h[dd_bucket(key, logB)], 1u);
        pk[slot] = key;
        pj[slot] = j;
    }
}

// One workgroup per bucket [hm[b G], hm[(b+1) G]): the keys go into an LDS
// table (a repeated key sets the duplicate mark), then each pair reads its
// key's mark into dupf[j].  A bucket with more distinct keys than a pass
// takes is done again in Q = 2, 4, ... passes, pass q taking the keys whose
// second hash is q mod Q (so a pass holds about 1/Q of them; copies of one
// key always share a pass).
__global__ __launch_bounds__(DD_NT) void k_dd_bucket(const u32 *hm, u32 G, u32 NB, const u64 *pk, const u32 *pj,
                                                     u8 *dupf, u32 *err)
{
    __shared__ u64 tab[DD_TSLOTS];
    __shared__ u32 s_new, s_over;
    for (u32 b = blockIdx.x; b < NB; b += gridDim.x) {
        const u32 e0 = hm[(u64)b * G], e1 = hm[(u64)(b + 1) * G];
        if (e0 >= e1) continue;  // (uniform)
        for (u32 Q = 1;; Q *= 2) {
            if (Q > (1u << 24)) {  // (keys of one class share a 24-bit second hash: never in practice)
                if (threadIdx.x == 0) atomicOr(err, 1u);
                break;
            }
            bool over = false;
            for (u32 q = 0; q < Q; q++) {
                for (u32 t = threadIdx.x; t < DD_TSLOTS; t += DD_NT) tab[t] = TAB_EMPTY;
                if (threadIdx.x == 0) {
                    s_new = 0;
                    s_over = 0;
                }
                __syncthreads();
                for (u32 e = e0 + threadIdx.x; e < e1; e += DD_NT) {
                    const u64 key = pk[e];
                    if (Q > 1 && dd_sub(key) % Q != q) continue;
                    u32 sl = dd_slot(key);
                    for (;;) {  // (at most DD_CAP + DD_NT keys: the table never fills)
                        u64 cur = tab[sl];
                        if (cur == TAB_EMPTY) {
                            if (__hip_atomic_load(&s_over, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) break;
                            cur = atomicCAS((unsigned long long *)&tab[sl], TAB_EMPTY, key);
                            if (cur == TAB_EMPTY) {
                                if (atomicAdd(&s_new, 1u) >= DD_CAP) atomicOr(&s_over, 1u);
                                break;
                            }
                        }
                        if ((cur & ~TAB_DUP) == key) {
                            if (!(cur & TAB_DUP)) atomicOr((unsigned long long *)&tab[sl], TAB_DUP);
                            break;
                        }
                        sl = (sl + 1) & (DD_TSLOTS - 1);
                    }
                }
                __syncthreads();
                if (s_over) {  // (uniform) too many keys for one pass: more passes
                    over = true;
                    __syncthreads();
                    break;
                }
                for (u32 e = e0 + threadIdx.x; e < e1; e += DD_NT) {
                    const u64 key = pk[e];
                    if (Q > 1 && dd_sub(key) % Q != q) continue;
                    u32 sl = dd_slot(key);
                    u8 d = 0;
                    for (;;) {
                        const u64 v = tab[sl];
                        if ((v & ~TAB_DUP) == key) {
                            d = (v & TAB_DUP) ? 1 : 0;
                            break;
                        }
                        if (v == TAB_EMPTY) break;  // (cannot happen: every key of the pass was inserted)
                        sl = (sl + 1) & (DD_TSLOTS - 1);
                    }
                    dupf[pj[e]] = d;
                }
                __syncthreads();
            }
            if (!over) break;
        }
    }
}

// Finish the active strings whose key is unique (or whose length is <= l):
// dist = min(len, l).  The others are appended to the next active list, with
// their key for the next round when a two-round pass computed it.  Each
// workgroup takes DD_PER x 256 list entries (lanes on consecutive entries)
// and reserves its part of the next list with one atomic: every reservation
// on that one counter is a round trip to the point where the chip's L2s meet,
// and they queue, so fewer and larger reservations.  Lists keep input order
// within a workgroup.
#define DD_PER 8

__global__ __launch_bounds__(256) void k_dedup(const u64 *keys, int kin, const u32 *act, const u32 *cnt,
                                               const u64 *off, u64 l, int mode, u32 *dist, u32 *next, u32 *ncnt,
                                               const u64 *carry, u64 *carry_out, const u8 *dupf)
{
    __shared__ u32 wcount[DD_PER][4], base;
    const u32 A = *cnt;
    const u32 lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const u32 j0 = blockIdx.x * (256u * DD_PER);
    u32 iq[DD_PER];
    u64 bq[DD_PER];
#pragma unroll
    for (u32 q = 0; q < DD_PER; q++) {
        const u32 j = j0 + q * 256 + threadIdx.x;
        bool stay = false;
        u32 i = 0;
        if (j < A) {
            i = act ? act[j] : j;
            const u64 len = off[i + 1] - off[i];
            const bool dup = mode == DM_ALLDUP || (mode == DM_TABLE && dupf[j] != 0);
            stay = dup && len > l;
            if (!stay) dist[i] = (u32)(len < l ? len : l);
        }
        iq[q] = i;
        bq[q] = __ballot(stay);
        if (lane == 0) wcount[q][w] = (u32)__popcll(bq[q]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 t = 0;
        for (u32 q = 0; q < DD_PER; q++) t += wcount[q][0] + wcount[q][1] + wcount[q][2] + wcount[q][3];
        base = t ? atomicAdd(ncnt, t) : 0u;
    }
    __syncthreads();
    u32 oq = base;  // first slot of row q (rows in list order, wavefronts in order within a row)
#pragma unroll
    for (u32 q = 0; q < DD_PER; q++) {
        u32 o = oq;
        for (u32 k = 0; k < w; k++) o += wcount[q][k];
        if ((bq[q] >> lane) & 1) {
            const u32 slot = o + (u32)__popcll(bq[q] & lanemask_lt());
            next[slot] = iq[q];
            if (carry) carry_out[slot] = carry[j0 + q * 256 + threadIdx.x];  // next round's key, already computed
        }
        oq += wcount[q][0] + wcount[q][1] + wcount[q][2] + wcount[q][3];
    }
}

// hdr: words 0..7 hold the u32 counters, 8..28 the flags of the precomputed
// rounds (three per round), 29 the first pass's deep decision, 30..35 the
// flags of a hash launch (rounds l and 2l); the host reads them back together.
#define HDR_WORDS 40
#define HDR_FIRST 8
#define HDR_DEEP (HDR_FIRST + 3 * PRE_ALL)
#define HDR_ROUND (HDR_DEEP + 1)
#define HDR_PRECOUNT (HDR_ROUND + 6)  // rounds the first pass precomputed (for a later rounds call)
#define HDR_CERT (HDR_PRECOUNT + 1)    // lazy deep pass: every string's certified LCP with string 0
#define HDR_MINLEN (HDR_CERT + 1)      // ... the shortest length
#define HDR_LAZY (HDR_MINLEN + 1)      // 1: the deep pass left its rounds of <= 64 bytes unhashed
struct PdWs {
    u32 *actA, *actB, *ctr;
    u64 *hdr, *keys, *keysB, *keysC, *state, *pre, *tab;
    v4i *wt;
    u32 *ddh, *ddscr;  // bucketed duplicate detection: counts matrix and its scan scratch
    u8 *dupt;          // table form: a duplicate mark per list position
};
#define CTR_DDERR 6  // ctr word: a bucket pass gave up (never in practice)

// Entries of the counts matrix (buckets x workgroups) the workspace holds.
static u64 dd_hm_cap(u64 n) { return (u64)DD_HM_CAP < 4 * n + 64 ? (u64)DD_HM_CAP : 4 * n + 64; }

// Whether a table round over Ah keys takes the bucketed form (tuning: 0 the
// global table, 1 buckets for lists of DD_MIN_ACT..DD_MAX_ACT keys, 2 buckets
// for every list up to DD_MAX_ACT).  On the 16M-string D/N step the two forms
// take the same time beside the sort, and the table alone is faster, so the
// table is the default.
static bool dd_use(u32 Ah)
{
    if (g_dedup_mode == 0) return false;
    if (g_dedup_mode == 2) return Ah <= DD_MAX_ACT;
    return Ah >= DD_MIN_ACT && Ah <= DD_MAX_ACT;
}

// Duplicate flags of the Ah active keys by buckets (see k_dd_count); the
// pairs and flags live in the (unused) global table's memory: keys 8 B, list
// positions 4 B and flags 1 B per entry within its >= 16 B per string.
static int dd_run(const u64 *keys, int kin, const u32 *act, const u32 *cntp, u32 Ah, u64 n, PdWs &w,
                  const u8 **dupf_out, hipStream_t st)
{
    const u64 cap = dd_hm_cap(n);
    u32 logB = 0;  // buckets of about 2048 keys
    if (g_dedup_logb > 0) logB = (u32)g_dedup_logb;
    else
        while (((u64)2048 << logB) < Ah && logB < DD_MAXLOG) logB++;
    while (logB > 0 && ((u64)1 << logB) > cap) logB--;
    const u32 NB = 1u << logB;
    // workgroups over chunks of >= 8192 entries, the matrix within its cap
    u64 G = ceil_div(Ah, 8192);
    if (G > cap / NB) G = cap / NB;
    if (G < 1) G = 1;
    const u32 C = (u32)ceil_div(Ah, G);
    G = ceil_div(Ah, C);
    u64 *pk = w.tab;
    u32 *pj = (u32 *)(w.tab + n);
    u8 *dupf = (u8 *)(pj + n);
    {
        SS_PROF("k_dd_count", st, (double)Ah * (act ? 16.0 : 8.0));  // (list entry,) key
        k_dd_count<<<(unsigned)G, DD_NT, 0, st>>>(keys, kin, act, cntp, logB, C, (u32)G, w.ddh);
    }
    SS_CHECK_LAUNCH();
    SS_TRY(ss_scan_exclusive<u32>(w.ddh, w.ddh, (u64)NB * G, w.ddscr, st));
    {
        SS_PROF("k_dd_scatter", st, (double)Ah * (act ? 28.0 : 20.0));  // (list entry,) key in, pair out
        k_dd_scatter<<<(unsigned)G, DD_NT, 0, st>>>(keys, kin, act, cntp, logB, C, (u32)G, w.ddh, pk, pj);
    }
    SS_CHECK_LAUNCH();
    {
        SS_PROF("k_dd_bucket", st, (double)Ah * 13.0);  // pair in, flag out
        k_dd_bucket<<<NB < 2048 ? NB : 2048, DD_NT, 0, st>>>(w.ddh, (u32)G, NB, pk, pj, dupf, w.ctr + CTR_DDERR);
    }
    SS_CHECK_LAUNCH();
    *dupf_out = dupf;
    return SS_OK;
}

static u32 tab_log(u64 A)
{
    u32 lg = 10;
    while ((1ull << lg) < 2 * A) lg++;
    return lg;
}

static void pd_layout(u64 n, PdWs *w, WsArena *a, WsCounter *c)
{
#define PT(field, T, cnt)                       \
    do {                                         \
        if (a) w->field = a->take<T>(cnt);       \
        else c->take<T>(cnt);                    \
    } while (0)
    PT(actA, u32, n); PT(actB, u32, n); PT(hdr, u64, HDR_WORDS); PT(keys, u64, n); PT(keysB, u64, n);
    PT(keysC, u64, n); PT(state, u64, n);
    PT(pre, u64, (u64)PRE_ALL * n); PT(tab, u64, 1ull << tab_log(n)); PT(wt, v4i, WT_ROUND + WT_FIRST);
    const u64 hm = dd_hm_cap(n) + 1;
    PT(ddh, u32, hm); PT(ddscr, u32, ss_scan_scratch_elems<u32>(hm));
    PT(dupt, u8, n);
#undef PT
    if (a) w->ctr = (u32 *)w->hdr;
}

extern "C" size_t ss_dist_prefix_workspace(uint64_t n)
{
    WsCounter c;
    PdWs w;
    pd_layout(n, &w, nullptr, &c);
    return c.used;
}

static u64 host_mulmod(u64 a, u64 b) { return (u64)(((unsigned __int128)a * b) % KR_P); }

static u64 host_powmod(u64 a, u64 e)
{
    u64 r = 1;
    for (; e; e >>= 1, a = host_mulmod(a, a))
        if (e & 1) r = host_mulmod(r, a);
    return r;
}

// Weights of the first pass: inverse powers of the base (B^(p-2) = B^-1 by
// Fermat, p prime) and the offset corrections of each round.
static FirstW first_weights()
{
    FirstW f{};
    const u64 binv = host_powmod(KR_B, KR_P - 2);
    u64 x = binv;
    for (int j = 0; j < 16; j++, x = host_mulmod(x, binv)) f.ib[j] = x;
    return f;
}

// Weights of a later round: inverse powers for the LDS table, the chunk
// scale of the first step and the powers that turn G into Horner values.
static RoundW round_weights(u64 lprev, u64 l1, u64 l2)
{
    RoundW r{};
    const u64 binv = host_powmod(KR_B, KR_P - 2);
    u64 x = binv;
    for (int k = 0; k < 16; k++, x = host_mulmod(x, binv)) r.iblo[k] = x;
    const u64 b16 = host_powmod(binv, 16);
    u64 y = 1;
    for (int k = 0; k < 16; k++, y = host_mulmod(y, b16)) r.ibhi[k] = y;
    r.ib256 = host_powmod(binv, 256);
    r.ibc0 = host_powmod(r.ib256, (lprev & ~63ull) / 1024);
    r.bl1 = host_powmod(KR_B, l1 / 4 + 1);
    r.bl2 = l2 ? host_powmod(KR_B, l2 / 4 + 1) : 0;
    u64 z = KR_B;
    for (int k = 0; k < 32; k++, z = host_mulmod(z, z)) r.b2[k] = z;
    return r;
}

enum { FP_PROBE = 0, FP_PLAIN = 1, FP_DEEP = 2 };

// The first pass over all n strings: the keys of every round whose prefix
// length is at most PRE_MAX (and, in the deep form, of the two rounds after
// it) into w.pre (round r at pre[r n + i]), their flags into the header, and
// the running sum G at the last precomputed round into w.state.  mode: the
// probe decides between the plain and the deep form (FP_PROBE; the probe's
// count is read back), or the caller does.  P receives the precomputed
// lengths (count 0: init_len > PRE_MAX, nothing launched).
// Sort seed layout: a 256-byte header (word 0: 1 when the pass wrote the
// seed, 0 when it did not), then the 8 bytes of every string at its mismatch
// (u64, n), then its mismatch position and byte count there (uint2, n).
#define SEED_HDR 256

static int first_pass(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n, uint32_t init_len,
                      uint32_t hash_bits, PdWs &w, int mode, PreLens &P, hipStream_t st, void *seed = nullptr,
                      const u64 *set_off = nullptr, u32 nsets = 1, bool lazy_ok = false)
{
    if (seed) {  // not written unless the deep pass runs
        k_store_u32<<<1, 1, 0, st>>>((u32 *)seed, 0u);
        SS_CHECK_LAUNCH();
    }
    k_store_u64<<<1, 1, 0, st>>>(w.hdr + HDR_LAZY, 0ull);
    SS_CHECK_LAUNCH();
    P = PreLens{};
    for (u64 L = init_len; L <= PRE_MAX && P.count < PRE_SLOTS; L *= 2) P.l[P.count++] = L;
    if (!P.count) return SS_OK;
    BPow bp;
    bp.p[0] = 1;
    for (int t = 1; t < 32; t++) bp.p[t] = (u64)(((unsigned __int128)bp.p[t - 1] * KR_B) % KR_P);
    u64 *fl_first = w.hdr + HDR_FIRST;
    const u32 c0 = P.count;
    // the deep form also precomputes the two rounds after 64 bytes (128 and
    // 256) from the same read; it needs a round of exactly 64 bytes
    const bool deep_ok = P.l[c0 - 1] == PRE_MAX;
    const u64 tiles = ceil_div(n, 32);
    const unsigned blocks = (unsigned)(ceil_div(tiles, 4) < 2048 ? ceil_div(tiles, 4) : 2048);
    // the flags of every precomputed round, then the probe's count (zero)
    k_flag_init<<<1, 64, 0, st>>>(fl_first, 3 * PRE_ALL + 1, 3 * PRE_ALL);
    SS_CHECK_LAUNCH();
    bool deep = mode == FP_DEEP && deep_ok;
    if (mode == FP_PROBE && deep_ok) {
        // deep when a sample of the strings shows a long shared prefix; the
        // decision is read back so that only the chosen kernel is launched (an
        // idle launch beside other streams' work would still wait for room on
        // the compute units)
        const u32 S = n < DEEP_SAMPLE ? (u32)n : DEEP_SAMPLE;
        k_deep_probe<<<(S + 255) / 256, 256, 0, st>>>((u32)n, bytes, N, offsets, w.hdr + HDR_DEEP);
        SS_CHECK_LAUNCH();
        u64 cnt = 0;
        SS_TRY(ss_read_u64(w.hdr + HDR_DEEP, &cnt, 1, st));
        deep = deep_from_count(cnt, (u32)n);
    }
    PassArgs A{};
    A.n = (u32)n;
    A.bytes = bytes;
    A.N = N;
    A.off = offsets;
    A.lprev = 0;
    A.l1 = 2 * PRE_MAX;
    A.l2 = 4 * PRE_MAX;
    A.bits = hash_bits;
    A.state = w.state;
    A.pre = w.pre;
    A.fl = fl_first;
    FirstArgs Fa{};
    Fa.P = P;
    Fa.bp = bp;
    Fa.fw = first_weights();
    // (the pass keeps every set's first string in LDS: with more sets it
    // writes no seed, and the sort compares everything itself)
    if (set_off && nsets > SEED_MAX_SETS) {
        seed = nullptr;
        set_off = nullptr;  // (a lazy certificate then compares with string 0)
    }
    if (seed && deep) {
        Fa.seed_word = (u64 *)((u8 *)seed + SEED_HDR);
        Fa.seed_pos = (uint2 *)((u8 *)seed + SEED_HDR + 8 * n);
    }
    if (deep) {
        Fa.set_off = set_off;
        Fa.nsets = set_off ? nsets : 1u;
    }
    // Lazy: the deep pass leaves the rounds of <= 64 bytes out and certifies
    // instead how long a prefix every string shares with string 0; the rounds
    // call hashes them only if that does not show them unable to finish any
    // string.
    const bool lazy = deep && lazy_ok;
    if (lazy) {
        Fa.lazy = 1;
        Fa.cert = w.hdr + HDR_CERT;
        Fa.minlen = w.hdr + HDR_MINLEN;
        k_store_u64<<<1, 1, 0, st>>>(w.hdr + HDR_CERT, ~0ull);
        SS_CHECK_LAUNCH();
        k_store_u64<<<1, 1, 0, st>>>(w.hdr + HDR_MINLEN, ~0ull);
        SS_CHECK_LAUNCH();
        k_store_u64<<<1, 1, 0, st>>>(w.hdr + HDR_LAZY, 1ull);
        SS_CHECK_LAUNCH();
    }
    if (!deep) {
        // algorithmic bytes: each string's prefix read once, its offsets, one
        // key written per precomputed round
        SS_PROF("k_hash_first", st, (double)n * (double)P.l[c0 - 1] + (double)n * (8.0 + 8.0 * c0));
        k_hash_first<<<blocks, 256, 0, st>>>((u32)n, bytes, N, offsets, P, hash_bits, bp, Fa.fw, w.state, w.pre,
                                             fl_first, 1u);
        SS_CHECK_LAUNCH();
    } else {
        const RoundW rwd = round_weights(0, 2 * PRE_MAX, 4 * PRE_MAX);
        k_hash_weights<<<(WT_ROUND + WT_FIRST + 255) / 256, 256, 0, st>>>(rwd, Fa, w.wt);
        SS_CHECK_LAUNCH();
        A.wt = w.wt;
        // The lazy form usually runs alone (a seeded sort waits for its
        // seed): one wave of resident workgroups, each striding over many
        // tiles, leaves no tail of late workgroups (1.55 -> 1.45 ms at 16M
        // strings against 8192).  The deep form keeps more, shorter workgroups than the plain
        // pass: beside the other stream's kernels they give compute units
        // back sooner.
        const u64 wg4 = ceil_div(tiles, 4);
        const u64 cap = lazy ? (u64)resident(k_hash_first_lazy, 256) : 8192ull;
        const unsigned dblocks = (unsigned)(wg4 < cap ? wg4 : cap);
        const double dbytes = (double)n * (4.0 * PRE_MAX) + (double)n * (8.0 + 8.0 * (lazy ? 2 : c0 + 2) + (seed ? 16.0 : 0.0));
        if (lazy) {
            SS_PROF("k_hash_first_lazy", st, dbytes);
            k_hash_first_lazy<<<dblocks, 256, 0, st>>>(A, rwd, Fa);
        } else {
            SS_PROF("k_hash_first_deep", st, dbytes);
            k_hash_first_deep<<<dblocks, 256, 0, st>>>(A, rwd, Fa);
        }
        SS_CHECK_LAUNCH();
        if (seed) {
            k_store_u32<<<1, 1, 0, st>>>((u32 *)seed, 1u);
            SS_CHECK_LAUNCH();
        }
        P.l[c0] = 2 * PRE_MAX;
        P.l[c0 + 1] = 4 * PRE_MAX;
        P.count = c0 + 2;
    }
    return SS_OK;
}


enum { PD_FIRST = 1, PD_ROUNDS = 2 };

// Prefix doubling in two parts that share the workspace: PD_FIRST hashes the
// first pass (and leaves its flags and round count in the header), PD_ROUNDS
// runs the remaining rounds and the duplicate detection from there.
static int pd_run(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n, uint32_t init_len,
                  uint32_t hash_bits, uint32_t *dist_approx, uint32_t *rounds_host, void *ws, size_t ws_bytes,
                  void *stream, int parts, void *seed = nullptr, int fp_mode = FP_PROBE,
                  const u64 *set_off = nullptr, u32 nsets = 1)
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
    if (!offsets || (!dist_approx && (parts & PD_ROUNDS))) { ss_set_error("null pointer"); return SS_ERR_INVALID_ARG; }
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
    for (int t = 1; t < 32; t++) bp.p[t] = (u64)(((unsigned __int128)bp.p[t - 1] * KR_B) % KR_P);
    // counters: [0], [1] active-list lengths (current / next, swapped per
    // round), [2], [3] the round's flags, [4..] flags of the first-pass rounds
    u32 *ctr = w.ctr;
    u64 *fl_round = w.hdr + HDR_ROUND;
    // rounds whose prefix length is at most PRE_MAX are hashed in one first pass
    PreLens P{};
    u32 pf[2 * PRE_ALL] = {};
    if (parts & PD_FIRST) {
        k_store_u32<<<1, 1, 0, st>>>(ctr, (u32)n);
        SS_CHECK_LAUNCH();
        SS_TRY(first_pass(bytes, N, offsets, n, init_len, hash_bits, w, fp_mode, P, st, seed, set_off, nsets, true));
        k_store_u64<<<1, 1, 0, st>>>(w.hdr + HDR_PRECOUNT, P.count);
        SS_CHECK_LAUNCH();
        if (!(parts & PD_ROUNDS)) return SS_OK;
    }
    {
        // the flags of every precomputed round, (rounds call alone) their
        // count, and a lazy deep pass's certificate
        u64 F[HDR_LAZY + 1 - HDR_FIRST];
        SS_TRY(ss_read_u64(w.hdr + HDR_FIRST, F, HDR_LAZY + 1 - HDR_FIRST, st));
        if (!(parts & PD_FIRST)) {
            // the lengths follow from init_len and the count (plain pass: the
            // rounds up to 64 bytes; deep pass: and the two after)
            const u64 cnt = F[HDR_PRECOUNT - HDR_FIRST];
            P = PreLens{};
            for (u64 L = init_len; L <= PRE_MAX && P.count < PRE_SLOTS; L *= 2) P.l[P.count++] = L;
            if (cnt == (u64)P.count + 2) {
                P.l[P.count] = 2 * PRE_MAX;
                P.l[P.count + 1] = 4 * PRE_MAX;
                P.count += 2;
            } else if (cnt != P.count) {
                ss_set_error("the workspace holds no first pass for init_len %u", init_len);
                return SS_ERR_INVALID_ARG;
            }
        }
        for (u32 r = 0; r < P.count; r++) {
            pf[2 * r] = F[3 * r] != F[3 * r + 1];
            pf[2 * r + 1] = F[3 * r + 2] != 0;
        }
        if (F[HDR_LAZY - HDR_FIRST] && P.count >= 2) {
            // The deep pass hashed only the rounds after 64 bytes.  Every
            // string shares its first `cert` bytes with string 0 and is
            // `mlen` bytes long or longer: when both reach past the longest
            // of those rounds, each of them has one key for all and no short
            // string -- it finishes nothing, the list stays whole, and its
            // keys are never read.  Otherwise the plain pass hashes them now
            // (without touching the running sums of the deep pass).
            const u32 cs = P.count - 2;
            const u64 cert = F[HDR_CERT - HDR_FIRST], mlen = F[HDR_MINLEN - HDR_FIRST];
            const bool need = cs > 0 && (cert < P.l[cs - 1] || mlen <= P.l[cs - 1]);
            if (!need) {
                for (u32 r = 0; r < cs; r++) pf[2 * r] = pf[2 * r + 1] = 0;
            } else {
                PreLens Ps = P;
                Ps.count = cs;
                k_flag_init<<<1, 64, 0, st>>>(w.hdr + HDR_FIRST, 3 * cs, 3 * cs);
                SS_CHECK_LAUNCH();
                const u64 tiles = ceil_div(n, 32);
                const unsigned blocks = (unsigned)(ceil_div(tiles, 4) < 2048 ? ceil_div(tiles, 4) : 2048);
                SS_PROF("k_hash_first", st, (double)n * (double)Ps.l[cs - 1] + (double)n * (8.0 + 8.0 * cs));
                k_hash_first<<<blocks, 256, 0, st>>>((u32)n, bytes, N, offsets, Ps, hash_bits, bp, first_weights(),
                                                     w.state, w.pre, w.hdr + HDR_FIRST, 0u);
                SS_CHECK_LAUNCH();
                SS_TRY(ss_read_u64(w.hdr + HDR_FIRST, F, 3 * cs, st));
                for (u32 r = 0; r < cs; r++) {
                    pf[2 * r] = F[3 * r] != F[3 * r + 1];
                    pf[2 * r + 1] = F[3 * r + 2] != 0;
                }
            }
        }
    }
    k_store_u32<<<1, 1, 0, st>>>(ctr + CTR_DDERR, 0u);
    SS_CHECK_LAUNCH();
    bool dd_used = false;
    u32 Ah = (u32)n;           // active count (exact after each flag read)
    const u32 *act = nullptr;  // the active strings (NULL = all, in input order)
    u32 *nxt = w.actA;
    int ci = 0;                // which counter holds the current count
    u64 lprev = 0, l = init_len;
    u32 rounds = 0;
    bool last_trivial = false;  // the previous round finished no string
    // this round's keys (list order) from a two-round pass: written to keysB,
    // compacted into keysC when the round before them shrank the list
    const u64 *pend = nullptr;
    // flags of the pending round from the two-round launch, valid while the
    // list has not changed since (the round in between finished nothing)
    bool pend_flags = false;
    u32 pend_differ = 0, pend_shrt = 0;
    for (;;) {
        const u64 *keys;
        const u64 *pend_next = nullptr;
        int kin = 0;
        u64 lhashed = 0;  // prefix length of this round's hash launch (0: none)
        bool fused_flags = false;  // this round's flags come from the hash launch
        bool have_flags = false;   // ... or from the previous launch (pending round)
        u32 differ = 0, shrt = 0;
        if (rounds < P.count) {
            keys = w.pre + (u64)rounds * n;
            kin = 1;
        } else if (pend) {
            keys = pend;
            if (pend_flags) {
                have_flags = true;
                differ = pend_differ;
                shrt = pend_shrt;
            }
        } else {
            // When the previous round finished nothing, hash this round and the
            // next from one read (the next round's keys wait in keysB).
            // (the first round's key is read out at a 64-byte step boundary)
            const bool two = last_trivial && lprev > 0 && l % 64 == 0;
            {
                // bytes are charged once the active count is read back
                SS_PROF("k_hash_round", st, 0.0);
                const u64 tiles = ceil_div(Ah, 32);
                const u64 nb = ceil_div(tiles, 4);
                k_flag_init<<<1, 64, 0, st>>>(fl_round, 6, 6);
                PassArgs A{};
                A.act = act;
                A.cnt = ctr + ci;
                A.bytes = bytes;
                A.N = N;
                A.off = offsets;
                A.lprev = lprev;
                A.l1 = l;
                A.l2 = two ? 2 * l : 0;
                A.bits = hash_bits;
                A.state = w.state;
                A.keys1 = w.keys;
                A.keys2 = w.keysB;
                A.rf = fl_round;
                k_hash_round<<<(unsigned)(nb < 1024 ? (nb ? nb : 1) : 1024), 256, 0, st>>>(
                    A, round_weights(lprev, l, two ? 2 * l : 0));
            }
            SS_CHECK_LAUNCH();
            keys = w.keys;
            lhashed = two ? 2 * l : l;
            if (two) pend_next = w.keysB;
            fused_flags = true;
        }
        pend_flags = false;
        if (!act && rounds < P.count) {
            differ = pf[2 * rounds];
            shrt = pf[2 * rounds + 1];
        } else if (have_flags) {
            // pending round of a two-round launch over an unchanged list: Ah holds
        } else if (fused_flags) {
            // the counters and the launch's flags in one read-back
            u64 H[HDR_ROUND + 6];
            SS_TRY(ss_read_u64(w.hdr, H, HDR_ROUND + 6, st));
            const u32 *h = (const u32 *)H;
            Ah = h[ci];
            const u64 *R = H + HDR_ROUND;
            differ = R[0] != R[1];
            shrt = R[2] != 0;
            if (pend_next) {
                pend_flags = true;
                pend_differ = R[3] != R[4];
                pend_shrt = R[5] != 0;
            }
            if (Ah == 0) ss_prof_drop_last("k_hash_round");
            else
                ss_prof_add_bytes("k_hash_round", (double)Ah * (double)(lhashed - lprev) +
                                                      (double)Ah * (pend_next ? 52.0 : 44.0));
        } else {
            SS_HIP(hipMemsetAsync(ctr + 2, 0, 2 * sizeof(u32), st));
            k_flags<<<(unsigned)ceil_div(Ah, 256), 256, 0, st>>>(keys, kin, act, ctr + ci, offsets, l, ctr + 2);
            SS_CHECK_LAUNCH();
            u32 h[4];
            SS_TRY(ss_read_u32(ctr, h, 4, st));
            Ah = h[ci];
            differ = h[2];
            shrt = h[3];
            if (lhashed) {
                // new prefix bytes (exact for strings of length >= the prefix),
                // offsets, list entry, hash state in/out, keys out; a launch over an
                // empty list is not counted
                if (Ah == 0) ss_prof_drop_last("k_hash_round");
                else
                    ss_prof_add_bytes("k_hash_round", (double)Ah * (double)(lhashed - lprev) +
                                                          (double)Ah * (pend_next ? 52.0 : 44.0));
            }
        }
        pend = nullptr;
        if (Ah == 0) break;
        if (++rounds > 64) { ss_set_error("prefix doubling did not terminate"); return SS_ERR_INVALID_ARG; }
        if (Ah >= 2 && !differ && !shrt) {
            // one key shared by all and no short string: nothing finishes
            last_trivial = true;
            pend = pend_next;  // (its flags stay valid: the list is unchanged)
            lprev = l;
            l *= 2;
            continue;
        }
        last_trivial = false;
        pend_flags = false;  // this round changes the list
        const int mode = Ah == 1 ? DM_UNIQUE : (differ ? DM_TABLE : DM_ALLDUP);
        u32 logT = 0;
        const u8 *dupf = nullptr;
        if (mode == DM_TABLE && dd_use(Ah)) {
            SS_TRY(dd_run(keys, kin, act, ctr + ci, Ah, n, w, &dupf, st));
            dd_used = true;
        } else if (mode == DM_TABLE) {
            logT = tab_log(Ah);
            SS_HIP(hipMemsetAsync(w.tab, 0xFF, sizeof(u64) << logT, st));
            SS_HIP(hipMemsetAsync(w.dupt, 0, Ah, st));
            {
                SS_PROF("k_tab_insert", st, (double)Ah * 28.0);  // list entry, key, slot read + write
                k_tab_insert<<<(unsigned)ceil_div(Ah, 256), 256, 0, st>>>(keys, kin, act, ctr + ci, w.tab, logT,
                                                                          w.dupt);
            }
            SS_CHECK_LAUNCH();
            dupf = w.dupt;
        }
        SS_HIP(hipMemsetAsync(ctr + (ci ^ 1), 0, sizeof(u32), st));
        {
            // list entry, offsets, key, slot, dist or next entry (and a carried key)
            SS_PROF("k_dedup", st, (double)Ah * ((mode == DM_TABLE ? 25.0 : 24.0) + (pend_next ? 16.0 : 0.0)));
            k_dedup<<<(unsigned)ceil_div(Ah, 256 * DD_PER), 256, 0, st>>>(keys, kin, act, ctr + ci, offsets, l, mode,
                                                                 dist_approx, nxt, ctr + (ci ^ 1), pend_next,
                                                                 w.keysC, dupf);
        }
        SS_CHECK_LAUNCH();
        if (pend_next) pend = w.keysC;
        act = nxt;
        nxt = (nxt == w.actA) ? w.actB : w.actA;
        ci ^= 1;
        lprev = l;
        l *= 2;
        if (Ah >= (1u << 20)) {
            // a large list: read the new count now rather than launch the next
            // round over it blindly (a launch over ~A/64 workgroups that may all
            // find the list empty costs about as much as this read-back)
            SS_TRY(ss_read_u32(ctr + ci, &Ah, 1, st));
            if (Ah == 0) break;
        }
    }
    if (dd_used) {
        u32 e = 0;
        SS_TRY(ss_read_u32(ctr + CTR_DDERR, &e, 1, st));
        if (e) {
            ss_set_error("duplicate detection: a bucket's keys did not split into passes");
            return SS_ERR_INVALID_ARG;
        }
    }
    if (rounds_host) *rounds_host = rounds;
    return SS_OK;
}

extern "C" int ss_dist_prefix(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                              uint32_t init_len, uint32_t hash_bits, uint32_t *dist_approx,
                              uint32_t *rounds_host, void *ws, size_t ws_bytes, void *stream)
{
    return pd_run(bytes, N, offsets, n, init_len, hash_bits, dist_approx, rounds_host, ws, ws_bytes, stream,
                  PD_FIRST | PD_ROUNDS);
}

extern "C" int ss_dist_prefix_first(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                    uint32_t init_len, uint32_t hash_bits, void *ws, size_t ws_bytes, void *stream)
{
    return pd_run(bytes, N, offsets, n, init_len, hash_bits, nullptr, nullptr, ws, ws_bytes, stream, PD_FIRST);
}

extern "C" size_t ss_sort_seed_bytes(uint64_t n) { return SEED_HDR + 16 * (size_t)n; }

extern "C" int ss_dist_prefix_first_seed(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                         const uint64_t *set_off, uint32_t num_sets, uint32_t init_len,
                                         uint32_t hash_bits, uint32_t first_pass_mode, void *sort_seed, void *ws,
                                         size_t ws_bytes, void *stream)
{
    if (!sort_seed || first_pass_mode > FP_DEEP || (set_off && num_sets == 0)) {
        ss_clear_error();
        ss_set_error(!sort_seed ? "null sort_seed"
                                : (first_pass_mode > FP_DEEP ? "first_pass_mode must be 0, 1 or 2" : "num_sets is 0"));
        return SS_ERR_INVALID_ARG;
    }
    return pd_run(bytes, N, offsets, n, init_len, hash_bits, nullptr, nullptr, ws, ws_bytes, stream, PD_FIRST,
                  sort_seed, (int)first_pass_mode, set_off, num_sets);
}

extern "C" int ss_dist_prefix_rounds(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                     uint32_t init_len, uint32_t hash_bits, uint32_t *dist_approx,
                                     uint32_t *rounds_host, void *ws, size_t ws_bytes, void *stream)
{
    return pd_run(bytes, N, offsets, n, init_len, hash_bits, dist_approx, rounds_host, ws, ws_bytes, stream,
                  PD_ROUNDS);
}

// The keys of the first `rounds` doubling rounds for every string, as the
// rounds of ss_dist_prefix compute them (first pass, then round passes), with
// every string kept active: keys[t n + i] = key of s_i[0, min(l_t, len)).
extern "C" int ss_doubling_keys(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                uint32_t init_len, uint32_t hash_bits, uint32_t rounds, uint32_t first_pass_mode,
                                uint64_t *keys, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (init_len == 0 || (init_len % 4) != 0) {
        ss_set_error("init_len must be a positive multiple of 4");
        return SS_ERR_INVALID_ARG;
    }
    if (hash_bits < 8 || hash_bits > 64) { ss_set_error("hash_bits must be 8..64"); return SS_ERR_INVALID_ARG; }
    if (first_pass_mode > FP_DEEP) { ss_set_error("first_pass_mode must be 0, 1 or 2"); return SS_ERR_INVALID_ARG; }
    if (rounds > 32 || ((u64)init_len << (rounds ? rounds - 1 : 0)) > (1ull << 31)) {
        ss_set_error("too many rounds");
        return SS_ERR_INVALID_ARG;
    }
    if (n == 0 || rounds == 0) return SS_OK;
    if (!offsets || !keys) { ss_set_error("null pointer"); return SS_ERR_INVALID_ARG; }
    hipStream_t st = (hipStream_t)stream;
    WsArena a(ws, ws_bytes);
    PdWs w;
    pd_layout(n, &w, &a, nullptr);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_dist_prefix_workspace(n));
        return SS_ERR_WORKSPACE;
    }
    PreLens P{};
    SS_TRY(first_pass(bytes, N, offsets, n, init_len, hash_bits, w, (int)first_pass_mode, P, st));
    u32 t = 0;
    for (; t < P.count && t < rounds; t++)
        SS_HIP(hipMemcpyAsync(keys + (u64)t * n, w.pre + (u64)t * n, sizeof(u64) * n, hipMemcpyDeviceToDevice, st));
    // the rounds after the first pass hash every string; two rounds per
    // launch where the round kernel allows it (as after a round that finished
    // nothing), so that both launch forms are exercised
    k_store_u32<<<1, 1, 0, st>>>(w.ctr, (u32)n);
    SS_CHECK_LAUNCH();
    u64 lprev = P.count ? P.l[P.count - 1] : 0;
    u64 l = (u64)init_len << t;
    while (t < rounds) {
        const bool two = lprev > 0 && l % 64 == 0 && t + 1 < rounds;
        k_flag_init<<<1, 64, 0, st>>>(w.hdr + HDR_ROUND, 6, 6);
        SS_CHECK_LAUNCH();
        PassArgs A{};
        A.act = nullptr;
        A.cnt = w.ctr;
        A.bytes = bytes;
        A.N = N;
        A.off = offsets;
        A.lprev = lprev;
        A.l1 = l;
        A.l2 = two ? 2 * l : 0;
        A.bits = hash_bits;
        A.state = w.state;
        A.keys1 = keys + (u64)t * n;
        A.keys2 = two ? keys + (u64)(t + 1) * n : nullptr;
        A.rf = w.hdr + HDR_ROUND;
        const u64 nb = ceil_div(ceil_div(n, 32), 4);
        k_hash_round<<<(unsigned)(nb < 1024 ? nb : 1024), 256, 0, st>>>(A, round_weights(lprev, l, two ? 2 * l : 0));
        SS_CHECK_LAUNCH();
        const u32 done = two ? 2 : 1;
        lprev = l << (done - 1);
        l <<= done;
        t += done;
    }
    return SS_OK;
}
