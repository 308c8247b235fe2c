// Segmented MSD radix string sort with LCP by-product (gfx950).
//
// Sorting the local string array is the first step of the paper's merge sort
// (Section 3, "Initialization"); the LCP array is its by-product.  This is a
// GPU-native design, not the paper's CPU algorithm:
//
//   * The sorted array is a set of contiguous SEGMENTS whose strings share a
//     known prefix of `depth` bytes.  Segment boundaries are final.
//   * Each ROUND takes the unresolved segments and
//       1. skips their common prefix: every string is compared with the
//          segment's first string from `depth` on and the minimum LCP is added
//          to `depth` (deep shared prefixes cost one read of D bytes, not one
//          radix pass per 7 bytes);
//       2. loads a 64-bit key per string: the next 7 bytes big-endian plus the
//          remaining length capped at 8, so that integer order is string order
//          over that window, end-of-string below every byte;
//       3. sorts each segment by (key, input index): segments larger than the
//          LDS cutover go through MSD byte passes (histogram, global scan,
//          stable scatter); segments of up to 128 strings are sorted by one
//          wavefront each with a bitonic network in registers; the others are
//          packed into LDS tiles and sorted by a bitonic network in LDS;
//       4. where neighbours' keys differ the LCP is final and is written; runs
//          of equal keys whose strings continue become next round's segments
//          at depth + 7; runs of equal keys whose strings end are equal
//          strings (LCP = length, order = input index).
#include <string.h>

#include "common.hpp"
#include <map>
#include <mutex>

#include "sort_core.hpp"

#define NT 256
#define ETILE 2048  // elements per workgroup in element-wise round kernels
#define RX_PF 8     // 256-element chunks a radix pass loads ahead
#define LDS_NT 512
#define LDS_CAP 2048  // elements per LDS tile (2 x the largest cutover)

// counters: list lengths, and the tile / element totals of the lists being
// built (so that grids are known without reading the lists back)
enum {
    C_SMALL = 0, C_LARGE = 1, C_NEXT = 2, C_IDENT = 3, C_BND = 4,
    C_LTILES = 5, C_SMALLN = 6, C_NTILES = 7, C_ITILES = 8, C_LELEM = 9, C_NELEM = 12, C_TINY = 13,
    C_TINYN = 14, C_BADSET = 15, C_NCTR = 16
};
// Headers that the round and level kernels read their list lengths from
// (copied from the counters by k_round_begin / k_level_begin, so that the
// counters can be reset for the lists being built): hdr[H_ACT] active
// segments, hdr[H_LARGE] radix segments of the current level, hdr[H_HIST]
// their histogram length (256 per tile).
enum { H_ACT = 0, H_LARGE = 1, H_HIST = 2, H_REMAIN = 3, H_NHDR = 4 };
#define WS_MAX 128  // segments of up to this many strings: one wavefront each
// ctr[10..11]: 64-bit sum of size * skip over the routed segments

// ------------------------------------------------------------ wave helpers

// Wave-aggregated atomic add of per-lane values.
__device__ __forceinline__ void wave_add(u32 v, u32 *counter)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (__lane_id() == 0 && v) atomicAdd(counter, v);
}

__device__ __forceinline__ u32 seg_of_tile(const u32 *tstart, u32 nseg, u32 t)
{
    // largest s with tstart[s] <= t (tstart has nseg+1 entries, strictly
    // increasing).  Every segment has a tile, so s <= t, and all but
    // extra = tstart[nseg] - nseg segments have one, so s >= t - extra: with
    // many small segments (one tile each) the search is short.
    const u32 extra = tstart[nseg] - nseg;
    u32 lo = t > extra ? t - extra : 0u;
    u32 hi = (t < nseg - 1 ? t : nseg - 1) + 1;
    while (hi - lo > 1) {
        u32 mid = (lo + hi) >> 1;
        if (tstart[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <class T, int NTB = NT>
__device__ __forceinline__ T block_min(T v)
{
    __shared__ T red[NTB / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T y = __shfl_xor(v, o, 64);
        v = y < v ? y : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = red[0];
    for (int w = 1; w < NTB / 64; w++) r = red[w] < r ? red[w] : r;
    __syncthreads();
    return r;
}

template <class T>
__device__ __forceinline__ T block_max(T v)
{
    __shared__ T red[NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T y = __shfl_xor(v, o, 64);
        v = y > v ? y : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = red[0];
    for (int w = 1; w < NT / 64; w++) r = red[w] > r ? red[w] : r;
    __syncthreads();
    return r;
}

// ------------------------------------------------------------ tile lists

// Every kernel below reads the length of the list it works on from device
// memory and takes its items in a grid-stride loop, so one launch shape
// serves any length: the host either sizes the grid from counts it read back,
// or launches a fixed grid without reading anything back.

#define GSTRIDE(j, count) for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < (count); j += gridDim.x * blockDim.x)

// Tile loop of the heavier kernels: with LOOP, a grid-stride loop over `count`
// tiles (fixed grids); without, exactly one tile per workgroup, t = blockIdx.x
// (grids sized from counts read back) -- the loop then runs once and compiles
// away, keeping the kernel's registers as they were.
#define TILE_LOOP(t, count) \
    for (u32 t = blockIdx.x; LOOP ? (t < (count)) : (t == blockIdx.x); t += LOOP ? gridDim.x : 1u)

__global__ void k_tile_counts(const Seg *segs, const u32 *nsegp, u32 tile, u32 *out)
{
    const u32 nseg = *nsegp;
    GSTRIDE(j, nseg) out[j] = (segs[j].end - segs[j].begin + tile - 1) / tile;
}

// Start of a round: the active list's length goes to the header, the
// counters of the lists the round builds are reset.
__global__ void k_round_begin(u32 *ctr, u32 *hdr)
{
    if (threadIdx.x == 0) hdr[H_ACT] = ctr[C_NEXT];
    __syncthreads();
    if (threadIdx.x < C_NCTR && threadIdx.x != C_BADSET) ctr[threadIdx.x] = 0;
}

// Tile counts of the active segments for a round; also resets the segments'
// skip minima.
__global__ void k_round_tiles(const Seg *segs, const u32 *nsegp, u32 tile, u32 *out, u32 *skipv)
{
    const u32 nseg = *nsegp;
    GSTRIDE(j, nseg) {
        out[j] = (segs[j].end - segs[j].begin + tile - 1) / tile;
        skipv[j] = 0xFFFFFFFFu;
    }
}

// Start of a radix level: the radix list's length and its histogram length
// go to the header, the counters of the next level's radix list are reset.
__global__ void k_level_begin(u32 *ctr, u32 *hdr, u32 nb)
{
    if (threadIdx.x == 0) {
        hdr[H_LARGE] = ctr[C_LARGE];
        hdr[H_HIST] = nb * ctr[C_LTILES];
        ctr[C_LARGE] = 0;
        ctr[C_LTILES] = 0;
        ctr[C_LELEM] = 0;
    }
}

// Tile counts of the radix segments of a level; also resets their key minima
// and maxima.
__global__ void k_level_tiles(const Seg *segs, const u32 *nsegp, u32 tile, u32 *out, u64 *smin, u64 *smax)
{
    const u32 nseg = *nsegp;
    GSTRIDE(j, nseg) {
        out[j] = (segs[j].end - segs[j].begin + tile - 1) / tile;
        smin[j] = ~0ull;
        smax[j] = 0;
    }
}

__global__ void k_sizes(const Seg *segs, const u32 *nsegp, u32 *out)
{
    const u32 nseg = *nsegp;
    GSTRIDE(j, nseg) out[j] = segs[j].end - segs[j].begin;
}

// ------------------------------------------------------------ round kernels

#define SKB 16      // strings per wavefront batch in the skip kernel
#define SKC_LONG 17  // 16-byte chunks per string of a long window (covers >= 257 bytes)
#define SKC_SHORT 5  // ... of a short window (covers >= 65 bytes)
#define SKR 5120     // LDS bytes per wavefront: five 1 KiB transfer rows
#define SKFS 256     // words (8 bytes) of the segment's first string staged in LDS

typedef __attribute__((address_space(3))) void lds_void;

// 8 bytes (little-endian) at any byte offset of LDS, from aligned words.
__device__ __forceinline__ u64 lds_le8(const u8 *R, u32 a)
{
    const u32 *p = (const u32 *)(R + (a & ~3u));
    const u32 r = a & 3u;
    u64 v = (u64)p[0] | ((u64)p[1] << 32);
    if (r) v = (v >> (8 * r)) | ((u64)p[2] << (64 - 8 * r));
    return v;
}

__device__ __forceinline__ u64 mask_le(u64 v, u32 take) { return take >= 8 ? v : (v & ((1ull << (8 * take)) - 1ull)); }

// Copy the window chunks of the batch's strings into the wavefront's LDS rows:
// chunk c of string s (16 bytes at the string's 16-aligned window start wa[s]
// plus 16c, relative to `bytes`) goes to R + 16 (CH s + c); wn[s] chunks are
// copied (0 for a window reaching outside the byte array, which is compared
// from global memory instead).
template <int CH>
__device__ __forceinline__ void skip_copy(const u8 *bytes, u8 *R, u32 lane, const u64 *wa, const u32 *wn)
{
    constexpr int T = (SKB * CH + 63) / 64;
    u64 ad[T];
    bool ok[T];
#pragma unroll
    for (int t = 0; t < T; t++) {  // every address first: the copies then issue back to back
        u32 slot = 64 * t + lane;
        asm volatile("" : "+v"(slot));  // recomputed per window rather than held in registers
        const u32 s = slot / CH, c = slot % CH;
        ad[t] = wa[s & 15] + 16u * c;
        ok[t] = s < SKB && c < wn[s & 15];
    }
#pragma unroll
    for (int t = 0; t < T; t++)
        if (ok[t]) __builtin_amdgcn_global_load_lds((const void *)(bytes + ad[t]), (lds_void *)(R + 1024 * t), 16, 0, 0);
}

// First mismatch of a member with the first string in [x, lim): each of the
// member's four lanes compares words q, q+4, q+8, ... (8 bytes each) of the
// window.  Returns the position (~0 if none) after a minimum over the four.
// Positions are string-relative (strings are shorter than 2^32 bytes).
template <int CH>
__device__ __forceinline__ u32 skip_cmp(const u8 *bytes, u64 N, const u8 *R, const u64 *fsw, u32 s, u32 q,
                                        u32 x, u32 lim, u32 sh, bool edge, u64 o, u64 fo, u32 depth)
{
    constexpr int WPL = (16 * CH + 31) / 32;  // words per lane
    const u32 rl = lim - x;                    // window bytes to compare (<= 16 CH)
    const u32 k0 = (x - depth) >> 3;           // first-string word of the window start
    const u32 rb = 16 * CH * s + sh;           // LDS offset of the window start
    u32 best = 0xFFFFFFFFu;
#pragma unroll 3
    for (int k = 0; k < WPL; k++) {
        const u32 w = q + 4 * k;
        const u32 rel = 8 * w;
        const u32 take = rel < rl ? ((rl - rel) < 8 ? rl - rel : 8u) : 0u;
        u64 wa = 0, wb = 0;
        if (take) {
            wa = edge ? load_le(bytes, N, o + x + rel, take) : mask_le(lds_le8(R, rb + rel), take);
            const u32 kw = k0 + w;
            wb = kw < SKFS ? mask_le(fsw[kw], take) : load_le(bytes, N, fo + x + rel, take);
        }
        const u64 d = wa ^ wb;
        const u32 mp = d ? rel + (u32)(__builtin_ctzll(d) >> 3) : 0xFFFFFFFFu;
        best = mp < best ? mp : best;
    }
#pragma unroll
    for (int o2 = 1; o2 < 4; o2 <<= 1) {
        const u32 y = __shfl_xor(best, o2, 64);
        best = y < best ? y : best;
    }
    return best == 0xFFFFFFFFu ? best : x + best;
}

// Minimum LCP of every member with the segment's first string, from `depth`.
// Each wavefront takes its members 16 at a time, four lanes per member: the
// window of every member (a short one of >= 65 bytes, or a long one of >= 257
// bytes once most members of the previous batch reached past 48 bytes) is
// copied from global memory into LDS by the transfer unit, then the four lanes
// compare it, 8 bytes at a time, against the first string's bytes
// [depth, depth + 2048) in LDS.  Members not resolved inside their window
// continue with the next one.  Each member also leaves its first mismatch
// position, its remaining length there (capped at 8) and its 8 bytes there
// (mword, mpr), from which k_keys builds its key without reading the string
// again.
//
// SEED (the first round of a seeded sort, one segment from depth 0 in input
// order): when *seed_ok, mword and mpr arrive holding every member's record
// as far as an earlier pass over the first bytes found it; a member whose
// mpr.y is SEED_OPEN agreed with the first string up to mpr.x and is compared
// from there, every other one is done without reading its string.
#define SEED_OPEN 0xFFFFFFFFu
// (the grid-stride form keeps its loop state live as well: five workgroups
// per compute unit give it the registers to do so without spilling)
template <bool LOOP, bool SEED = false, int NTB = NT>
__global__ __launch_bounds__(NTB, (LOOP ? 5 : 6) * (NT / NTB)) void k_skip(const Seg *segs, const u32 *tstart, const u32 *nsegp,
                                             const u8 *bytes, u64 N, const u64 *off,
                                             const u32 *perm, u32 *skipv, u64 *mword, uint2 *mpr,
                                             const u32 *seed_ok = nullptr)
{
    __shared__ u64 fsw[SKFS];
    __shared__ __attribute__((aligned(16))) u8 rows[(NTB / 64) * SKR];
    __shared__ u64 wwa[NTB / 64][SKB];  // per wavefront: window start of each member
    __shared__ u32 wwn[NTB / 64][SKB];  // ... and its chunk count
    const u32 nseg = *nsegp;
    const u32 ntiles = LOOP ? tstart[nseg] : 0u;
    const bool sok = SEED && *seed_ok != 0;  // uniform
    TILE_LOOP(t, ntiles) {  // (uniform over the workgroup)
    const u32 sg = seg_of_tile(tstart, nseg, t);
    const Seg g = segs[sg];
    if (!(g.aux & SEG_SKIP)) continue;  // uniform over the workgroup
    const u32 lt = t - tstart[sg];
    const u32 b0 = g.begin + lt * ETILE;
    const u32 b1 = min(g.end, b0 + ETILE);
    if (SEED && sok) {
        // the tile's records, one member per thread: when the seed resolved
        // every member, their minimum is the tile's part of the skip and no
        // string is read (a tile with an open member takes the loop below)
        u32 sb = 0xFFFFFFFFu;
        bool open = false;
#pragma unroll 8
        for (u32 k = 0; k < ETILE / NTB; k++) {
            const u32 i = b0 + k * NTB + threadIdx.x;
            if (i < b1) {
                const uint2 sp = mpr[i];
                open |= sp.y == SEED_OPEN;
                const u32 c = sp.x > g.depth ? sp.x - g.depth : 0u;
                sb = c < sb ? c : sb;
            }
        }
        if (!__syncthreads_or(open)) {  // (uniform)
            const u32 bm = block_min<u32, NTB>(sb);
            if (threadIdx.x == 0) atomicMin(&skipv[sg], bm);
            continue;
        }
    }
    const u32 f = perm[g.begin];
    const u64 fo = off[f];
    const u32 fl = (u32)(off[f + 1] - fo);
    const u32 depth = g.depth;
    const u32 fd = fl > depth ? fl - depth : 0;  // first-string bytes from depth
    for (u32 q = threadIdx.x; q < SKFS; q += NTB) {
        const u32 k = 8 * q;
        fsw[q] = k < fd ? load_le(bytes, N, fo + depth + k, (fd - k) < 8 ? fd - k : 8u) : 0ull;
    }
    __syncthreads();
    const u32 lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const u32 sl = lane >> 2, q = lane & 3;  // this lane's member of the batch, its quarter
    u8 *R = rows + wv * SKR;
    const u64 babs = (u64)(uintptr_t)bytes;
    bool longw = false;  // window size of the next batch (uniform over the wavefront)
    u32 best = 0xFFFFFFFFu;
    for (u32 i0 = b0 + wv * SKB; i0 < b1; i0 += (NTB / 64) * SKB) {
        const u32 i = i0 + sl;
        const bool valid = i < b1;
        u64 o = 0;
        u32 len = 0, m = 0, x = depth;
        bool seeded = false;  // done by the seed
        u32 sres = 0;
        if (SEED && sok && valid) {
            const uint2 sp = mpr[i];
            if (sp.y != SEED_OPEN) {
                seeded = true;
                sres = sp.x;
            } else {
                x = sp.x;
            }
        }
        if (valid && !seeded) {
            const u32 p = perm[i];
            o = off[p];
            len = (u32)(off[p + 1] - o);
            m = len < fl ? len : fl;
        }
        u32 res = seeded ? sres : m;
        bool act = valid && !seeded && x < m;
        while (__ballot(act)) {  // uniform over the wavefront
            const u32 CH = longw ? SKC_LONG : SKC_SHORT;
            const u64 A0 = (babs + o + x) & ~15ull;
            const u32 sh = (u32)((babs + o + x) & 15);
            const u32 cov = 16 * CH - sh;                      // window bytes from x
            const u32 wend = len - x < cov ? len : x + cov;    // copied: [x, wend)
            const u32 lim = m - x < cov ? m : x + cov;         // compared: [x, lim)
            const u32 nch = act ? (sh + (wend - x) + 15) / 16 : 0u;
            // a window reaching outside the byte array is compared from global memory
            const bool edge = act && (A0 < babs || A0 + 16ull * nch > babs + N);
            if (q == 0) {  // (read back below by the same wavefront: LDS keeps its order)
                wwa[wv][sl] = A0 - babs;
                wwn[wv][sl] = edge ? 0u : nch;
            }
            u32 mis;
            if (longw) {
                skip_copy<SKC_LONG>(bytes, R, lane, wwa[wv], wwn[wv]);
                mis = skip_cmp<SKC_LONG>(bytes, N, R, fsw, sl, q, x, act ? lim : x, sh, edge, o, fo, depth);
            } else {
                skip_copy<SKC_SHORT>(bytes, R, lane, wwa[wv], wwn[wv]);
                mis = skip_cmp<SKC_SHORT>(bytes, N, R, fsw, sl, q, x, act ? lim : x, sh, edge, o, fo, depth);
            }
            if (act) {
                u32 r = mis;
                if (r == 0xFFFFFFFFu && lim >= m) r = m;
                if (r != 0xFFFFFFFFu) {
                    // the member's 8 bytes at its mismatch, from the window when it holds them
                    const u32 rem = len - r;
                    const u32 tk = rem < 8 ? rem : 8u;
                    if (q == 0) {
                        u64 mw = 0;
                        if (tk)
                            mw = (!edge && r + tk <= wend) ? mask_le(lds_le8(R, 16 * CH * sl + sh + (r - x)), tk)
                                                           : load_le(bytes, N, o + r, tk);
                        mword[i] = __builtin_bswap64(mw);
                        mpr[i] = make_uint2(r, tk);
                    }
                    res = r;
                    act = false;
                } else {
                    x += cov & ~7u;
                }
            }
        }
        // most of the batch reaching past 48 bytes from depth: long windows next
        const bool far = valid && res >= depth + 48;
        longw = __popcll(__ballot(far && q == 0)) >= SKB / 2;
        if (valid && q == 0) {
            const u32 c = res > depth ? res - depth : 0u;
            best = c < best ? c : best;
            if (!seeded && m <= depth) {  // nothing to compare: the member ends at or before depth
                const u32 rem = len - res;
                const u32 tk = rem < 8 ? rem : 8u;
                mword[i] = load_be(bytes, N, o + res, tk);
                mpr[i] = make_uint2(res, tk);
            }
        }
    }
    const u32 bm = block_min<u32, NTB>(best);  // (ends with a barrier: fsw and the rows are free again)
    if (threadIdx.x == 0) atomicMin(&skipv[sg], bm);
    }
}

template <bool LOOP, int NTB = NT>
__global__ __launch_bounds__(NTB) void k_keys(const Seg *segs, const u32 *tstart, const u32 *nsegp,
                                             const u8 *bytes, u64 N, const u64 *off,
                                             const u32 *perm, const u32 *skipv, const u64 *mword,
                                             const uint2 *mpr, u64 *keys)
{
    __shared__ u64 fw;
    const u32 nseg = *nsegp;
    const u32 ntiles = LOOP ? tstart[nseg] : 0u;
    TILE_LOOP(t, ntiles) {
    const u32 s = seg_of_tile(tstart, nseg, t);
    const Seg g = segs[s];
    const u32 lt = t - tstart[s];
    const u32 b0 = g.begin + lt * ETILE;
    const u32 b1 = min(g.end, b0 + ETILE);
    if (!(g.aux & SEG_SKIP)) {
        const u64 d = g.depth;
        for (u32 i = b0 + threadIdx.x; i < b1; i += NTB) {
            const u32 p = perm[i];
            const u64 o = off[p], l = off[p + 1] - o;
            keys[i] = make_key(bytes, N, o, l, d);
        }
        continue;  // (uniform over the workgroup)
    }
    // A member agrees with the segment's first string up to its mismatch
    // position pos >= d, so its key at d is the first string's bytes [d, pos)
    // followed by its own bytes from pos (mword).
    const u64 d = (u64)g.depth + skipv[s];
    if (threadIdx.x == 0) {
        const u32 f = perm[g.begin];
        const u64 fo = off[f], fl = off[f + 1] - fo;
        const u64 r = fl - d;  // the first string is a member: fl >= d
        fw = load_be(bytes, N, fo + d, r < 7 ? (u32)r : 7u);
    }
    __syncthreads();
    for (u32 i = b0 + threadIdx.x; i < b1; i += NTB) {
        const uint2 pr = mpr[i];
        const u32 k = pr.x - (u32)d;  // bytes shared with the first string beyond d
        u64 data = fw;
        if (k < 7) {
            const u64 keep = k ? (~0ull << (64 - 8 * k)) : 0ull;
            data = (fw & keep) | (mword[i] >> (8 * k));
        }
        const u32 cnt = pr.y + k < 8 ? pr.y + k : 8u;
        keys[i] = (data & ~0xFFull) | cnt;
    }
    __syncthreads();  // fw is rewritten by the next tile
    }
}

// Apply the skip, route each active segment to the LDS list or the radix list.
__global__ void k_classify(const Seg *act, const u32 *nactp, const u32 *skipv, u32 small_max, u32 tile, Seg *tiny,
                           Seg *small, Seg *large, u32 *ctr)
{
    const u32 nact = *nactp;
    for (u32 j0 = blockIdx.x * blockDim.x; j0 < nact; j0 += gridDim.x * blockDim.x) {
    const u32 j = j0 + threadIdx.x;
    bool valid = j < nact;
    Seg g = {0, 0, 0, 0};
    if (valid) {
        g = act[j];
        if (g.aux & SEG_SKIP) g.depth += skipv[j];
        g.aux = 0;
    }
    const bool ty = valid && (g.end - g.begin) <= WS_MAX;
    const bool sm = valid && !ty && (g.end - g.begin) <= small_max;
    const bool lg = valid && !ty && !sm;
    const u32 c = wave_append(ty, &ctr[C_TINY]);
    if (ty) tiny[c] = g;
    u32 a = wave_append(sm, &ctr[C_SMALL]);
    if (sm) small[a] = g;
    u32 b = wave_append(lg, &ctr[C_LARGE]);
    if (lg) large[b] = g;
    const u32 sz = g.end - g.begin;
    {
        u64 sk = (valid && (act[j].aux & SEG_SKIP)) ? (u64)sz * skipv[j] : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sk += __shfl_xor(sk, o, 64);
        if (__lane_id() == 0 && sk) atomicAdd((unsigned long long *)&ctr[10], (unsigned long long)sk);
    }
    wave_add(ty ? sz : 0u, &ctr[C_TINYN]);
    wave_add(sm ? sz : 0u, &ctr[C_SMALLN]);
    wave_add(lg ? (sz + tile - 1) / tile : 0u, &ctr[C_LTILES]);
    wave_add(lg ? sz : 0u, &ctr[C_LELEM]);
    }
}

// ------------------------------------------------------------ radix passes
//
// A radix level sorts a segment by one digit of the 64-bit key.  The digit
// width W is 8 bits (eight levels per key, one per byte) or 11 bits (six
// levels: five of 11 bits and a last one of 9 that ends with the key's
// length byte).  Level l covers key bits [lo, hi) with hi = 64 - W l and
// lo = max(0, hi - W); its histograms have 2^W buckets.

template <u32 W>
struct Digits {
    static constexpr u32 NB = 1u << W;                 // buckets of a level
    static constexpr u32 LEVELS = (64 + W - 1) / W;    // levels of one key
    static constexpr u32 DPT = NB / 256;               // digits per thread of a 256-thread workgroup
};

template <u32 W>
__device__ __forceinline__ u32 digit_of(u64 k, u32 level)
{
    const u32 hi = 64 - W * level;
    const u32 lo = hi > W ? hi - W : 0u;
    return (u32)(k >> lo) & ((1u << (hi - lo)) - 1u);
}

// Lanes of this wave holding the same W-bit digit (restricted to `valid`).
template <u32 W>
__device__ __forceinline__ u64 match_digit_w(u32 digit, bool valid)
{
    u64 m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < (int)W; b++) {
        u64 bb = __ballot((digit >> b) & 1);
        m &= ((digit >> b) & 1) ? bb : ~bb;
    }
    return m;
}

// Per-tile histogram of the segment's current digit, digit-major per
// segment: hist[NB*tstart[s] + d*T_s + lt].  Also the segment's min and max key.
template <bool LOOP, u32 W>
__global__ __launch_bounds__(NT) void k_hist(const Seg *segs, const u32 *tstart, const u32 *nsegp, u32 tile,
                                             const u64 *keyA, const u64 *keyB, u32 *hist, u64 *smin, u64 *smax)
{
    constexpr u32 NB = Digits<W>::NB;
    __shared__ u32 h[NB];
    const u32 nseg = *nsegp;
    const u32 ntiles = LOOP ? tstart[nseg] : 0u;
    TILE_LOOP(t, ntiles) {
    const u32 s = seg_of_tile(tstart, nseg, t);
    const Seg g = segs[s];
    const u64 *keys = (g.aux & SEG_INB) ? keyB : keyA;
    const u32 T = tstart[s + 1] - tstart[s];
    const u32 lt = t - tstart[s];
    const u32 level = g.aux & 15;
    const u32 b0 = g.begin + lt * tile;
    const u32 b1 = min(g.end, b0 + tile);
    for (u32 d = threadIdx.x; d < NB; d += NT) h[d] = 0;
    __syncthreads();
    u64 mn = ~0ull, mx = 0;
    for (u32 c0 = b0; c0 < b1; c0 += RX_PF * NT) {
        // RX_PF chunks' keys loaded before any is counted
        u64 kq[RX_PF];
#pragma unroll
        for (u32 q = 0; q < RX_PF; q++) {
            const u32 i = c0 + q * NT + threadIdx.x;
            kq[q] = i < b1 ? keys[i] : 0;
        }
#pragma unroll
        for (u32 q = 0; q < RX_PF; q++) {
            const u32 c = c0 + q * NT;
            if (c >= b1) break;  // (uniform)
            const bool valid = c + threadIdx.x < b1;
            const u64 k = kq[q];
            u32 d = digit_of<W>(k, level);
            u64 peers = match_digit_w<W>(d, valid);
            if (valid) {
                mn = k < mn ? k : mn;
                mx = k > mx ? k : mx;
                if ((peers & lanemask_lt()) == 0) atomicAdd(&h[d], (u32)__popcll(peers));
            }
        }
    }
    __syncthreads();
    for (u32 d = threadIdx.x; d < NB; d += NT) hist[NB * tstart[s] + d * T + lt] = h[d];
    mn = block_min(mn);
    mx = block_max(mx);  // (ends with a barrier: h is free again)
    if (threadIdx.x == 0) {
        atomicMin((unsigned long long *)&smin[s], (unsigned long long)mn);
        atomicMax((unsigned long long *)&smax[s], (unsigned long long)mx);
    }
    }
}

struct EmitOut {
    Seg *tiny, *small, *large_next, *next, *ident;
    uint2 *bnd;
    u32 *ctr;
    u8 *scat;
    u8 *kinds;
    u32 small_max;
    u32 tile;
};

enum { K_NONE = 0, K_SMALL, K_LARGE, K_NEXT, K_IDENT, K_TINY, K_KINDS };

// What digit d of radix segment s becomes: an entry for one of the lists
// (kind, seg) and/or a bucket boundary (sb, depth) for the LCP pass.
struct EmitItem {
    u32 kind;
    Seg ns;
    bool bnd;
    uint2 bv;
};

template <u32 W>
__device__ __forceinline__ EmitItem emit_item(const Seg *segs, const u32 *tstart, const u32 *hist, const u64 *smin,
                                              const u64 *smax, const EmitOut &o, u32 s, u32 d, bool *scat)
{
    constexpr u32 NB = Digits<W>::NB;
    EmitItem it{K_NONE, Seg{0, 0, 0, 0}, false, make_uint2(0, 0)};
    const Seg g = segs[s];
    const u32 level = g.aux & 15;
    const u32 pf = g.aux & SEG_INB;  // where the segment's data is now
    const u64 mn = smin[s], mx = smax[s];
    // next-round and equal-string runs (and singletons) end in A: the settle
    // pass copies them there; the other kinds carry their buffer flag
    if (mn == mx) {
        // one key for the whole segment (all 8 bytes): continue next round,
        // or equal strings
        *scat = false;
        const u32 cnt = (u32)(mn & 0xFF);
        if (d == 0) {
            if (cnt == 8) { it.kind = K_NEXT; it.ns = Seg{g.begin, g.end, g.depth + 7, SEG_SKIP}; }
            else { it.kind = K_IDENT; it.ns = Seg{g.begin, g.end, g.depth + cnt, 0}; }
        }
        return it;
    }
    const u32 fd = (u32)__clzll(mn ^ mx) / W;  // first digit where the keys differ
    if (fd > level) {
        // digits level..fd-1 are common to the whole segment: no scatter needed
        *scat = false;
        if (d == 0) { it.kind = K_LARGE; it.ns = Seg{g.begin, g.end, g.depth, fd | pf}; }
        return it;
    }
    *scat = true;
    const u32 cf = pf ? 0u : (u32)SEG_INB;  // the scatter writes the other arrays
    const u32 ts = tstart[s];
    const u32 T = tstart[s + 1] - ts;
    const u32 e = NB * ts + d * T;
    const u32 base = hist[NB * ts];
    const u32 start = hist[e] - base;
    const u32 cnt = hist[e + T] - hist[e];
    const u32 sb = g.begin + start, se = sb + cnt;
    it.bnd = cnt > 0 && start > 0;
    it.bv = make_uint2(sb, g.depth);
    it.ns = Seg{sb, se, g.depth, cf};
    if (cnt >= 2) {
        if (level == Digits<W>::LEVELS - 1) {
            // the last digit ends with the key's length byte: the bucket's
            // keys are equal in all 64 bits
            const u32 c8 = d & 0xFFu;
            if (c8 == 8) { it.kind = K_NEXT; it.ns = Seg{sb, se, g.depth + 7, SEG_SKIP}; }
            else { it.kind = K_IDENT; it.ns = Seg{sb, se, g.depth + c8, 0}; }
        } else if (cnt <= WS_MAX) {
            it.kind = K_TINY;
        } else if (cnt <= o.small_max) {
            it.kind = K_SMALL;
        } else {
            it.kind = K_LARGE;
            it.ns.aux = (level + 1) | cf;
        }
    }
    return it;
}

#define EPB 8  // emit items per thread in k_emit: 8 segments of 256 digits, or 1 segment of 2048

// Digit counts from the scanned histogram and emission of the sub-segments.
// A workgroup takes 8 / DPT segments (thread x = digits x + 256 r, r < DPT):
// it counts its entries in LDS, reserves room in every list with one global
// atomic per list, and then writes the entries.
template <bool LOOP, u32 W>
__global__ __launch_bounds__(256) void k_emit(const Seg *segs, const u32 *tstart, const u32 *nsegp,
                                              const u32 *hist, const u64 *smin, const u64 *smax,
                                              EmitOut o)
{
    constexpr u32 NB = Digits<W>::NB, DPT = Digits<W>::DPT, SPG = EPB / DPT;  // segments per group
    __shared__ u32 lcount[K_KINDS], lslot[K_KINDS], lsum[7], gbase[K_KINDS];
    const u32 nseg = *nsegp;
    const u32 ngrp = LOOP ? (nseg + SPG - 1) / SPG : 0u;
    TILE_LOOP(grp, ngrp) {
    const u32 s0 = grp * SPG;
    const u32 tx = threadIdx.x;
    if (tx < K_KINDS) { lcount[tx] = 0; lslot[tx] = 0; }
    if (tx < 7) lsum[tx] = 0;
    __syncthreads();
    EmitItem it[EPB];
#pragma unroll
    for (u32 q = 0; q < EPB; q++) {
        const u32 s = s0 + q / DPT;
        const u32 d = tx + 256u * (q % DPT);
        it[q].kind = K_NONE;
        it[q].bnd = false;
        if (s >= nseg) continue;
        bool sc = false;
        it[q] = emit_item<W>(segs, tstart, hist, smin, smax, o, s, d, &sc);
        if (d == 0) o.scat[s] = sc ? 1 : 0;
        o.kinds[NB * s + d] = (u8)it[q].kind;
        const EmitItem &x = it[q];
        const u32 cnt = x.ns.end - x.ns.begin;
        if (x.bnd) atomicAdd(&lcount[0], 1u);
        if (x.kind) atomicAdd(&lcount[x.kind], 1u);
        if (x.kind == K_SMALL) atomicAdd(&lsum[0], cnt);
        if (x.kind == K_LARGE) { atomicAdd(&lsum[1], (cnt + o.tile - 1) / o.tile); atomicAdd(&lsum[2], cnt); }
        if (x.kind == K_NEXT) { atomicAdd(&lsum[3], (cnt + ETILE - 1) / ETILE); atomicAdd(&lsum[4], cnt); }
        if (x.kind == K_IDENT) atomicAdd(&lsum[5], (cnt + ETILE - 1) / ETILE);
        if (x.kind == K_TINY) atomicAdd(&lsum[6], cnt);
    }
    __syncthreads();
    if (tx == 0) {
        gbase[0] = lcount[0] ? atomicAdd(&o.ctr[C_BND], lcount[0]) : 0u;
        gbase[K_SMALL] = lcount[K_SMALL] ? atomicAdd(&o.ctr[C_SMALL], lcount[K_SMALL]) : 0u;
        gbase[K_LARGE] = lcount[K_LARGE] ? atomicAdd(&o.ctr[C_LARGE], lcount[K_LARGE]) : 0u;
        gbase[K_NEXT] = lcount[K_NEXT] ? atomicAdd(&o.ctr[C_NEXT], lcount[K_NEXT]) : 0u;
        gbase[K_IDENT] = lcount[K_IDENT] ? atomicAdd(&o.ctr[C_IDENT], lcount[K_IDENT]) : 0u;
        gbase[K_TINY] = lcount[K_TINY] ? atomicAdd(&o.ctr[C_TINY], lcount[K_TINY]) : 0u;
        if (lsum[0]) atomicAdd(&o.ctr[C_SMALLN], lsum[0]);
        if (lsum[1]) atomicAdd(&o.ctr[C_LTILES], lsum[1]);
        if (lsum[2]) atomicAdd(&o.ctr[C_LELEM], lsum[2]);
        if (lsum[3]) atomicAdd(&o.ctr[C_NTILES], lsum[3]);
        if (lsum[4]) atomicAdd(&o.ctr[C_NELEM], lsum[4]);
        if (lsum[5]) atomicAdd(&o.ctr[C_ITILES], lsum[5]);
        if (lsum[6]) atomicAdd(&o.ctr[C_TINYN], lsum[6]);
    }
    __syncthreads();
#pragma unroll
    for (u32 q = 0; q < EPB; q++) {
        const EmitItem &x = it[q];
        if (x.bnd) o.bnd[gbase[0] + atomicAdd(&lslot[0], 1u)] = x.bv;
        if (x.kind) {
            const u32 a = gbase[x.kind] + atomicAdd(&lslot[x.kind], 1u);
            Seg *dst = x.kind == K_TINY ? o.tiny : x.kind == K_SMALL ? o.small
                     : x.kind == K_LARGE ? o.large_next : x.kind == K_NEXT ? o.next : o.ident;
            dst[a] = x.ns;
        }
    }
    __syncthreads();  // the LDS counters are reset for the next group
    }
}

// Stable scatter of (key, payload) by the current digit into the other pair
// of arrays (A -> B or B -> A, by the segment's flag).  run[d] is the next
// free position of digit d; in each chunk of NT elements the wavefronts take
// turns (wave 0 first, so that equal digits keep the input order), and in a
// wave the first lane of each digit reserves that digit's slots for all its
// peers; the others take the base from it by a shuffle.  The work per chunk
// does not grow with the number of buckets.
template <bool LOOP, u32 W>
__global__ __launch_bounds__(NT) void k_scatter(const Seg *segs, const u32 *tstart, const u32 *nsegp, u32 tile,
                                                const u32 *hist, const u8 *scat, u64 *keyA, u32 *valA,
                                                u64 *keyB, u32 *valB)
{
    constexpr u32 NB = Digits<W>::NB;
    __shared__ u32 run[NB];
    const u32 nseg = *nsegp;
    const u32 ntiles = LOOP ? tstart[nseg] : 0u;
    TILE_LOOP(t, ntiles) {
    const u32 s = seg_of_tile(tstart, nseg, t);
    if (!scat[s]) continue;  // (uniform over the workgroup)
    const Seg g = segs[s];
    const bool inb = g.aux & SEG_INB;
    const u64 *ksrc = inb ? keyB : keyA;
    const u32 *vsrc = inb ? valB : valA;
    u64 *kdst = inb ? keyA : keyB;
    u32 *vdst = inb ? valA : valB;
    const u32 ts = tstart[s];
    const u32 T = tstart[s + 1] - ts;
    const u32 lt = t - ts;
    const u32 level = g.aux & 15;
    const u32 b0 = g.begin + lt * tile;
    const u32 b1 = min(g.end, b0 + tile);
    const u32 base = hist[NB * ts];
    for (u32 d = threadIdx.x; d < NB; d += NT) run[d] = g.begin + hist[NB * ts + d * T + lt] - base;
    __syncthreads();
    const u32 wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (u32 c0 = b0; c0 < b1; c0 += RX_PF * NT) {
    // RX_PF chunks' keys and payloads loaded before any is placed
    u64 kq[RX_PF];
    u32 vq[RX_PF];
#pragma unroll
    for (u32 q = 0; q < RX_PF; q++) {
        const u32 i = c0 + q * NT + threadIdx.x;
        kq[q] = 0;
        vq[q] = 0;
        if (i < b1) {
            kq[q] = ksrc[i];
            vq[q] = vsrc[i];
        }
    }
#pragma unroll
    for (u32 q = 0; q < RX_PF; q++) {
        const u32 c = c0 + q * NT;
        if (c >= b1) break;  // (uniform)
        const u32 i = c + threadIdx.x;
        const bool valid = i < b1;
        const u64 k = kq[q];
        const u32 v = vq[q];
        const u32 d = digit_of<W>(k, level);
        const u64 peers = match_digit_w<W>(d, valid);
        const u32 rank = (u32)__popcll(peers & lanemask_lt());
        u32 slot = 0;
#pragma unroll
        for (u32 w = 0; w < NT / 64; w++) {
            if (wid == w && valid && rank == 0) {
                slot = run[d];
                run[d] = slot + (u32)__popcll(peers);
            }
            __syncthreads();
        }
        const int leader = valid ? __ffsll((unsigned long long)peers) - 1 : (int)lane;
        const u32 dst = __shfl(slot, leader, 64) + rank;
        if (valid) {
            kdst[dst] = k;
            vdst[dst] = v;
        }
    }
    }
    __syncthreads();  // run is rewritten by the next tile
    }
}

// After a level: buckets that no later kernel rewrites (singletons, runs for
// the next round, equal strings) are copied to A when the level left them in
// B.  Scattered segments read back their digits to find them; an unscattered
// segment that became such a run is copied whole.
template <bool LOOP, u32 W>
__global__ __launch_bounds__(NT) void k_settle(const Seg *segs, const u32 *tstart, const u32 *nsegp, u32 tile,
                                               const u8 *scat, const u8 *kinds, const u64 *keyB,
                                               const u32 *valB, u64 *keyA, u32 *valA)
{
    const u32 nseg = *nsegp;
    const u32 ntiles = LOOP ? tstart[nseg] : 0u;
    TILE_LOOP(t, ntiles) {
    const u32 s = seg_of_tile(tstart, nseg, t);
    const Seg g = segs[s];
    const bool inb = g.aux & SEG_INB;
    const u32 level = g.aux & 15;
    const u32 lt = t - tstart[s];
    const u32 b0 = g.begin + lt * tile;
    const u32 b1 = min(g.end, b0 + tile);
    const u8 *kd = kinds + Digits<W>::NB * s;
    if (scat[s]) {
        if (inb) continue;  // scattered into A
        for (u32 c0 = b0; c0 < b1; c0 += RX_PF * NT) {
            // RX_PF chunks' keys, then their buckets' kinds, loaded before any is used
            u64 kq[RX_PF];
            u32 cq[RX_PF];
#pragma unroll
            for (u32 q = 0; q < RX_PF; q++) {
                const u32 i = c0 + q * NT + threadIdx.x;
                kq[q] = i < b1 ? keyB[i] : 0ull;
            }
#pragma unroll
            for (u32 q = 0; q < RX_PF; q++) cq[q] = kd[digit_of<W>(kq[q], level)];
#pragma unroll
            for (u32 q = 0; q < RX_PF; q++) {
                const u32 i = c0 + q * NT + threadIdx.x;
                const u32 c = cq[q];
                if (i < b1 && (c == K_NONE || c == K_NEXT || c == K_IDENT)) {
                    keyA[i] = kq[q];
                    valA[i] = valB[i];
                }
            }
        }
    } else if (inb && (kd[0] == K_NEXT || kd[0] == K_IDENT)) {
        for (u32 i = b0 + threadIdx.x; i < b1; i += NT) {
            keyA[i] = keyB[i];
            valA[i] = valB[i];
        }
    }
    }
}

__global__ void k_boundary(const uint2 *bnd, const u32 *nbp, const u64 *keys, u32 *lcp)
{
    const u32 nb = *nbp;
    GSTRIDE(j, nb) {
        const uint2 b = bnd[j];
        lcp[b.x] = key_lcp(keys[b.x - 1], keys[b.x], b.y);
    }
}

// Equal strings: LCP = their length for every member after the first.
template <bool LOOP>
__global__ __launch_bounds__(NT) void k_ident(const Seg *segs, const u32 *tstart, const u32 *nsegp, u32 *lcp)
{
    const u32 nseg = *nsegp;
    const u32 ntiles = LOOP ? tstart[nseg] : 0u;
    TILE_LOOP(t, ntiles) {
        const u32 s = seg_of_tile(tstart, nseg, t);
        const Seg g = segs[s];
        const u32 lt = t - tstart[s];
        const u32 b0 = g.begin + lt * ETILE;
        const u32 b1 = min(g.end, b0 + ETILE);
        for (u32 i = b0 + threadIdx.x; i < b1; i += NT)
            if (i > g.begin) lcp[i] = g.depth;
    }
}

// ------------------------------------------------------------- LDS sort

__device__ __forceinline__ bool lds_greater(u16 sa, u64 ka, u32 va, u16 sb, u64 kb, u32 vb)
{
    if (sa != sb) return sa > sb;
    if (ka != kb) return ka > kb;
    return va > vb;
}

// Small segments packed into tiles: tile t takes the segments whose start in
// the concatenated small-segment space lies in [t*H, (t+1)*H); with segment
// sizes <= H a tile holds < 2H elements.  Sorted by (segment, key, payload)
// with a bitonic network in LDS.
template <bool LOOP>
__global__ __launch_bounds__(LDS_NT) void k_lds_sort(const Seg *small, const u32 *pref, const u32 *nsmallp,
                                                     u32 H, u64 *keys, u32 *vals, const u64 *keyB,
                                                     const u32 *valB, u32 *lcp, Seg *next, u32 *ctr)
{
    __shared__ u64 skey[LDS_CAP];
    __shared__ u32 sval[LDS_CAP];
    __shared__ u16 sseg[LDS_CAP];
    __shared__ u32 spref[LDS_CAP / 2 + 1];
    __shared__ u32 sbeg[LDS_CAP / 2];
    __shared__ u32 sdep[LDS_CAP / 2];
    __shared__ u8 sinb[LDS_CAP / 2];
    __shared__ Seg nq[LDS_CAP / 2];  // next-round segments found in this tile
    __shared__ u32 nq_count, nq_tiles, nq_elems, nq_base;
    const u32 nsmall = *nsmallp;
    const u32 ntile = LOOP ? (pref[nsmall] + H - 1) / H : 0u;  // pref[nsmall]: strings in all small segments
    TILE_LOOP(t, ntile) {
    const u32 lo = t * H, hi = lo + H;
    // j0 = first segment with pref >= lo, j1 = first with pref >= hi
    u32 j0, j1;
    {
        u32 a = 0, b = nsmall;
        while (a < b) { u32 m = (a + b) >> 1; if (pref[m] < lo) a = m + 1; else b = m; }
        j0 = a;
        a = j0; b = nsmall;
        while (a < b) { u32 m = (a + b) >> 1; if (pref[m] < hi) a = m + 1; else b = m; }
        j1 = a;
    }
    if (j0 >= j1) continue;  // (uniform over the workgroup)
    const u32 ns = j1 - j0;
    const u32 base = pref[j0];
    const u32 cnt = pref[j1] - base;
    if (threadIdx.x == 0) { nq_count = 0; nq_tiles = 0; nq_elems = 0; }
    for (u32 k = threadIdx.x; k <= ns; k += LDS_NT) spref[k] = pref[j0 + k] - base;
    for (u32 k = threadIdx.x; k < ns; k += LDS_NT) {
        Seg g = small[j0 + k];
        sbeg[k] = g.begin;
        sdep[k] = g.depth;
        sinb[k] = (g.aux & SEG_INB) ? 1 : 0;
    }
    __syncthreads();
    u32 P = 2;
    while (P < cnt) P <<= 1;
    for (u32 e = threadIdx.x; e < P; e += LDS_NT) {
        if (e < cnt) {
            u32 a = 0, b = ns;  // largest k with spref[k] <= e
            while (b - a > 1) { u32 m = (a + b) >> 1; if (spref[m] <= e) a = m; else b = m; }
            const u32 pos = sbeg[a] + (e - spref[a]);
            skey[e] = sinb[a] ? keyB[pos] : keys[pos];  // read where the segment is, write A
            sval[e] = sinb[a] ? valB[pos] : vals[pos];
            sseg[e] = (u16)a;
        } else {
            skey[e] = ~0ull;
            sval[e] = 0xFFFFFFFFu;
            sseg[e] = 0xFFFF;
        }
    }
    __syncthreads();
    for (u32 k = 2; k <= P; k <<= 1) {
        for (u32 j = k >> 1; j > 0; j >>= 1) {
            for (u32 i = threadIdx.x; i < P / 2; i += LDS_NT) {
                const u32 x = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                const u32 y = x + j;
                const bool up = (x & k) == 0;
                const u16 sx = sseg[x], sy = sseg[y];
                const u64 kx = skey[x], ky = skey[y];
                const u32 vx = sval[x], vy = sval[y];
                if (lds_greater(sx, kx, vx, sy, ky, vy) == up) {
                    sseg[x] = sy; sseg[y] = sx;
                    skey[x] = ky; skey[y] = kx;
                    sval[x] = vy; sval[y] = vx;
                }
            }
            __syncthreads();
        }
    }
    for (u32 e = threadIdx.x; e < cnt; e += LDS_NT) {
        const u32 a = sseg[e];
        const u32 first = spref[a];
        const u32 pos = sbeg[a] + (e - first);
        const u64 kb = skey[e];
        vals[pos] = sval[e];
        keys[pos] = kb;
        if (e == first) continue;
        const u64 ka = skey[e - 1];
        const u32 dep = sdep[a];
        if (ka != kb) {
            lcp[pos] = key_lcp(ka, kb, dep);
            continue;
        }
        const u32 c8 = (u32)(kb & 0xFF);
        if (c8 < 8) {
            lcp[pos] = dep + c8;
            continue;
        }
        const bool last = (e + 1 == spref[a + 1]) || skey[e + 1] != kb;
        if (last) {
            u32 x = first, y = e;  // first index in [first, e] with key == kb
            while (x < y) { u32 m = (x + y) >> 1; if (skey[m] < kb) x = m + 1; else y = m; }
            const Seg ns{sbeg[a] + (x - first), pos + 1, dep + 7, SEG_SKIP};
            const u32 slot = atomicAdd(&nq_count, 1u);
            nq[slot] = ns;
            atomicAdd(&nq_tiles, (ns.end - ns.begin + ETILE - 1) / ETILE);
            atomicAdd(&nq_elems, ns.end - ns.begin);
        }
    }
    // publish this tile's next-round segments with one atomic per counter
    __syncthreads();
    if (threadIdx.x == 0 && nq_count) {
        nq_base = atomicAdd(&ctr[C_NEXT], nq_count);
        atomicAdd(&ctr[C_NTILES], nq_tiles);
        atomicAdd(&ctr[C_NELEM], nq_elems);
    }
    __syncthreads();
    for (u32 k = threadIdx.x; k < nq_count; k += LDS_NT) next[nq_base + k] = nq[k];
    __syncthreads();  // the LDS tables are rewritten by the next tile
    }
}

#define WS_SPB 16  // tiny segments per workgroup (4 wavefronts, 4 segments each)

__device__ __forceinline__ bool kv_greater(u64 ka, u32 va, u64 kb, u32 vb)
{
    return ka != kb ? ka > kb : va > vb;
}

// Bitonic compare-exchange of element e with the element j lanes away
// (j < 64) in a merge of size k: the lower index of an ascending pair keeps
// the smaller (key, payload).
__device__ __forceinline__ void ws_step(u64 &key, u32 &val, u32 e, u32 j, u32 k)
{
    const u64 pk = __shfl_xor(key, (int)j, 64);
    const u32 pv = __shfl_xor(val, (int)j, 64);
    const bool want_small = ((e & j) == 0) == ((e & k) == 0);
    if (want_small == kv_greater(key, val, pk, pv)) {
        key = pk;
        val = pv;
    }
}

// LCP of sorted element e (e >= 1) from its predecessor's key, as in the LDS
// sort; returns whether e is the last of a run of >= 2 equal full keys (a
// next-round segment).
__device__ __forceinline__ bool ws_finish(u32 e, u32 cnt, u64 ka, u64 kb, u64 kn, u32 dep, u32 *lcp_out)
{
    if (e == 0 || e >= cnt) return false;
    if (ka != kb) {
        *lcp_out = key_lcp(ka, kb, dep);
        return false;
    }
    const u32 c8 = (u32)(kb & 0xFF);
    if (c8 < 8) {
        *lcp_out = dep + c8;
        return false;
    }
    return e + 1 == cnt || kn != kb;
}

__device__ __forceinline__ u32 hibit(u64 m) { return 63u - (u32)__clzll(m); }

#define WS_DEEP 3  // further 7-byte keys a wavefront reads for runs of equal continuing keys

__device__ __forceinline__ bool rkv_greater(u32 ra, u64 ka, u32 va, u32 rb, u64 kb, u32 vb)
{
    return ra != rb ? ra > rb : (ka != kb ? ka > kb : va > vb);
}

// ws_step on (run start, key, payload)
__device__ __forceinline__ void ws_step3(u32 &rs, u64 &key, u32 &val, u32 e, u32 j, u32 k)
{
    const u32 pr = __shfl_xor(rs, (int)j, 64);
    const u64 pk = __shfl_xor(key, (int)j, 64);
    const u32 pv = __shfl_xor(val, (int)j, 64);
    const bool want_small = ((e & j) == 0) == ((e & k) == 0);
    if (want_small == rkv_greater(rs, key, val, pr, pk, pv)) {
        rs = pr;
        key = pk;
        val = pv;
    }
}

__device__ __forceinline__ bool shfl_down_b(bool b, u32 lane, bool from_next)
{
    const int d = __shfl_down((int)b, 1, 64);
    return lane < 63 ? d != 0 : from_next;
}

// Segments of 2..128 strings, one wavefront each: bitonic sort of
// (key, payload) in registers (element e = lane + 64 r, r = 0, 1), then LCPs.
// Runs of equal continuing keys are not sent to the next round at once: the
// wavefront reads their strings' next 7-byte keys (up to WS_DEEP times) and
// sorts every run again by (run, key, payload), writing the LCPs of the
// pairs each key separates; runs still tied then become next-round segments,
// collected per workgroup and published with one atomic per counter.  (Equal
// strings, common in text, so end inside the wavefront instead of costing a
// workgroup per run in the next round's skip and key passes.)
template <bool LOOP>
__global__ __launch_bounds__(256) void k_wave_sort(const Seg *tiny, const u32 *ntinyp, u64 *keys, u32 *vals,
                                                   const u64 *keyB, const u32 *valB, u32 *lcp, Seg *next, u32 *ctr,
                                                   const u8 *bytes, u64 N, const u64 *off)
{
    __shared__ Seg nq[WS_SPB * (WS_MAX / 2)];
    __shared__ u32 nq_count, nq_tiles, nq_elems, nq_base;
    const u32 ntiny = *ntinyp;
    const u32 ngrp = LOOP ? (ntiny + WS_SPB - 1) / WS_SPB : 0u;
    TILE_LOOP(grp, ngrp) {
    if (threadIdx.x == 0) { nq_count = 0; nq_tiles = 0; nq_elems = 0; }
    __syncthreads();
    const u32 lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const u32 e0 = lane, e1 = lane + 64;
    // This wavefront's segments: all descriptors first, and each segment's
    // keys and payload loaded while the previous one is being sorted.
    Seg gq[WS_SPB / 4];
#pragma unroll
    for (u32 q = 0; q < WS_SPB / 4; q++) {
        const u32 sidx = grp * WS_SPB + q * 4 + wv;
        gq[q] = sidx < ntiny ? tiny[sidx] : Seg{0, 0, 0, 0};
    }
    u64 nk0 = ~0ull, nk1 = ~0ull;
    u32 nv0 = 0xFFFFFFFFu, nv1 = 0xFFFFFFFFu;
    auto fetch = [&](const Seg &g) {
        const u32 cnt = g.end - g.begin;
        const u64 *ks = (g.aux & SEG_INB) ? keyB : keys;  // read where the segment is, write A
        const u32 *vs = (g.aux & SEG_INB) ? valB : vals;
        nk0 = ~0ull; nk1 = ~0ull; nv0 = 0xFFFFFFFFu; nv1 = 0xFFFFFFFFu;
        if (e0 < cnt) { nk0 = ks[g.begin + e0]; nv0 = vs[g.begin + e0]; }
        if (e1 < cnt) { nk1 = ks[g.begin + e1]; nv1 = vs[g.begin + e1]; }
    };
    fetch(gq[0]);
#pragma unroll
    for (u32 q = 0; q < WS_SPB / 4; q++) {
        const u32 sidx = grp * WS_SPB + q * 4 + wv;
        if (sidx >= ntiny) break;  // uniform over the wavefront
        const Seg g = gq[q];
        const u32 cnt = g.end - g.begin;
        u64 k0 = nk0, k1 = nk1;
        u32 v0 = nv0, v1 = nv1;
        if (q + 1 < WS_SPB / 4) fetch(gq[q + 1]);
        u32 P = 2;
        while (P < cnt) P <<= 1;
        for (u32 k = 2; k <= P; k <<= 1) {
            for (u32 j = k >> 1; j > 0; j >>= 1) {
                if (j == 64) {
                    // partner of e0 is e1 in the same lane (k == 128: ascending)
                    if (kv_greater(k0, v0, k1, v1)) {
                        const u64 tk = k0; k0 = k1; k1 = tk;
                        const u32 tv = v0; v0 = v1; v1 = tv;
                    }
                } else {
                    ws_step(k0, v0, e0, j, k);
                    if (P == 128) ws_step(k1, v1, e1, j, k);
                }
            }
        }
        if (e0 < cnt) keys[g.begin + e0] = k0;
        if (e1 < cnt) keys[g.begin + e1] = k1;
        // neighbours in sorted order
        const u64 k0_last = __shfl(k0, 63, 64), k1_first = __shfl(k1, 0, 64);
        const u64 up0 = __shfl_up(k0, 1, 64), up1 = __shfl_up(k1, 1, 64);
        const u64 dn0 = __shfl_down(k0, 1, 64), dn1 = __shfl_down(k1, 1, 64);
        const u64 pa0 = up0, pa1 = lane ? up1 : k0_last;
        const u64 nx0 = lane < 63 ? dn0 : k1_first, nx1 = dn1;
        u32 l0 = 0, l1 = 0;
        ws_finish(e0, cnt, pa0, k0, nx0, g.depth, &l0);
        ws_finish(e1, cnt, pa1, k1, nx1, g.depth, &l1);
        // LCP writes (skipped for the first element and for equal full keys)
        if (e0 >= 1 && e0 < cnt && !(pa0 == k0 && (k0 & 0xFF) == 8)) lcp[g.begin + e0] = l0;
        if (e1 < cnt && !(pa1 == k1 && (k1 & 0xFF) == 8)) lcp[g.begin + e1] = l1;
        const u64 le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        // tied with the predecessor: equal keys, both strings continue
        bool t0 = e0 >= 1 && e0 < cnt && pa0 == k0 && (k0 & 0xFF) == 8;
        bool t1 = e1 < cnt && pa1 == k1 && (k1 & 0xFF) == 8;
        u32 dep = g.depth;
        if (__ballot(t0 || t1)) {  // (uniform: most segments have no run of equal keys)
        for (u32 it = 0; it < WS_DEEP; it++) {
            // in a run: tied with the predecessor or the successor (e0's successor
            // is e0 + 1, lane 63's is e1 of lane 0); every lane shuffles first
            const bool f1 = __shfl((int)t1, 0, 64) != 0;
            const bool n0 = shfl_down_b(t0, lane, f1), n1 = shfl_down_b(t1, lane, false);
            const bool in0 = t0 || n0, in1 = t1 || n1;
            if (!__ballot(in0 || in1)) break;  // (uniform)
            dep += 7;
            // run of every element: its first position (padding sorts last)
            const u64 s0 = __ballot(!t0), s1 = __ballot(!t1);
            const u64 ms = s1 & le;
            u32 rs0 = e0 < cnt ? hibit(s0 & le) : 0xFFFFFFFFu;
            u32 rs1 = e1 < cnt ? (ms ? 64u + hibit(ms) : hibit(s0)) : 0xFFFFFFFFu;
            u64 q0 = e0 < cnt ? 0ull : ~0ull, q1 = e1 < cnt ? 0ull : ~0ull;
            if (in0) {
                const u64 o = off[v0];
                q0 = make_key(bytes, N, o, off[v0 + 1] - o, dep);
            }
            if (in1) {
                const u64 o = off[v1];
                q1 = make_key(bytes, N, o, off[v1 + 1] - o, dep);
            }
            for (u32 k = 2; k <= P; k <<= 1) {
                for (u32 j = k >> 1; j > 0; j >>= 1) {
                    if (j == 64) {
                        if (rkv_greater(rs0, q0, v0, rs1, q1, v1)) {
                            const u32 tr = rs0; rs0 = rs1; rs1 = tr;
                            const u64 tq = q0; q0 = q1; q1 = tq;
                            const u32 tv = v0; v0 = v1; v1 = tv;
                        }
                    } else {
                        ws_step3(rs0, q0, v0, e0, j, k);
                        if (P == 128) ws_step3(rs1, q1, v1, e1, j, k);
                    }
                }
            }
            const u32 rp0 = __shfl_up(rs0, 1, 64), rl0 = __shfl(rs0, 63, 64), ru1 = __shfl_up(rs1, 1, 64);
            const u32 rp1 = lane ? ru1 : rl0;
            const u64 qp0 = __shfl_up(q0, 1, 64), ql0 = __shfl(q0, 63, 64), qu1 = __shfl_up(q1, 1, 64);
            const u64 qp1 = lane ? qu1 : ql0;
            const bool same0 = e0 >= 1 && e0 < cnt && rp0 == rs0;  // same run as the predecessor
            const bool same1 = e1 < cnt && rp1 == rs1;
            t0 = same0 && qp0 == q0 && (q0 & 0xFF) == 8;
            t1 = same1 && qp1 == q1 && (q1 & 0xFF) == 8;
            if (same0 && !t0) lcp[g.begin + e0] = qp0 != q0 ? key_lcp(qp0, q0, dep) : dep + (u32)(q0 & 0xFF);
            if (same1 && !t1) lcp[g.begin + e1] = qp1 != q1 ? key_lcp(qp1, q1, dep) : dep + (u32)(q1 & 0xFF);
        }
        // still tied: the last element of each run publishes it for the next round
        const bool f1 = __shfl((int)t1, 0, 64) != 0;
        const bool n0 = shfl_down_b(t0, lane, f1), n1 = shfl_down_b(t1, lane, false);
        const bool end0 = t0 && !n0, end1 = t1 && !n1;
        const u64 s0 = __ballot(!t0), s1 = __ballot(!t1);
        if (end0) {
            const u32 f = hibit(s0 & le);
            const Seg ns{g.begin + f, g.begin + e0 + 1, dep + 7, SEG_SKIP};
            nq[atomicAdd(&nq_count, 1u)] = ns;
            atomicAdd(&nq_tiles, (ns.end - ns.begin + ETILE - 1) / ETILE);
            atomicAdd(&nq_elems, ns.end - ns.begin);
        }
        if (end1) {
            const u64 mm = s1 & le;
            const u32 f = mm ? 64u + hibit(mm) : hibit(s0);
            const Seg ns{g.begin + f, g.begin + e1 + 1, dep + 7, SEG_SKIP};
            nq[atomicAdd(&nq_count, 1u)] = ns;
            atomicAdd(&nq_tiles, (ns.end - ns.begin + ETILE - 1) / ETILE);
            atomicAdd(&nq_elems, ns.end - ns.begin);
        }
        }
        if (e0 < cnt) vals[g.begin + e0] = v0;
        if (e1 < cnt) vals[g.begin + e1] = v1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && nq_count) {
        nq_base = atomicAdd(&ctr[C_NEXT], nq_count);
        atomicAdd(&ctr[C_NTILES], nq_tiles);
        atomicAdd(&ctr[C_NELEM], nq_elems);
    }
    __syncthreads();
    for (u32 k = threadIdx.x; k < nq_count; k += 256) next[nq_base + k] = nq[k];
    __syncthreads();  // nq and its counters are reset for the next group
    }
}

// ------------------------------------------------------------ host driver

void sort_ws_layout(u64 n, SortWs *w, WsArena *a, WsCounter *c)
{
    // Capacities: segments hold >= 2 strings (<= n/2 of them); radix segments
    // hold > 128 strings; radix tiles <= n/1024 + radix segments.
    const u64 nseg = n / 2 + 2;
    const u64 nlarge = n / 128 + 2;
    const u64 ntiles = n / 1024 + nlarge + 2;
    // histograms and bucket kinds: 256 buckets per radix tile / segment with
    // 8-bit digits; 2048 with 11-bit digits, which are used only with tiles
    // of >= 4096 and radix segments of > 512 strings
    const u64 nlarge11 = n / 512 + 2, ntiles11 = n / 4096 + nlarge11 + 2;
    const u64 nhist = 256 * ntiles > 2048 * ntiles11 ? 256 * ntiles : 2048 * ntiles11;
    const u64 nkinds = 256 * nlarge > 2048 * nlarge11 ? 256 * nlarge : 2048 * nlarge11;
    const u64 nscan = (nhist > nseg + 1 ? nhist : nseg + 1) + 1;
#define TAKE(field, T, cnt)                      \
    do {                                          \
        if (a) w->field = a->take<T>(cnt);        \
        else c->take<T>(cnt);                     \
    } while (0)
    TAKE(keyA, u64, n);
    TAKE(keyB, u64, n);
    TAKE(mword, u64, n);
    TAKE(mpr, uint2, n);
    TAKE(valB, u32, n);
    TAKE(lcp_scratch, u32, n);
    TAKE(act, Seg, nseg);
    TAKE(nxt, Seg, nseg);
    TAKE(tiny, Seg, nseg);
    TAKE(small, Seg, nseg);
    TAKE(ident, Seg, nseg);
    TAKE(largeA, Seg, nlarge);
    TAKE(largeB, Seg, nlarge);
    TAKE(bnd, uint2, n + 1);
    TAKE(skipv, u32, nseg);
    TAKE(smin, u64, nlarge);
    TAKE(smax, u64, nlarge);
    TAKE(scat, u8, nlarge);
    TAKE(kinds, u8, nkinds);
    TAKE(tstart, u32, nseg + 1);
    TAKE(spref, u32, nseg + 1);
    TAKE(hist, u32, nscan);
    TAKE(scan_scratch, u64, ss_scan_scratch_elems<u64>(nscan));
    TAKE(dscan, u32, ss_scan_dev_scratch_elems<u32>());
    TAKE(ctr, u32, C_NCTR);
    TAKE(hdr, u32, H_NHDR);
#undef TAKE
}

// Launch shapes.  A kernel over a list takes its items in a grid-stride loop;
// the host sizes its grid from the list's length when it knows it (read back),
// otherwise it launches a fixed grid bounded by the largest list possible.
static unsigned grid_of(u64 items, u64 per, u64 cap)
{
    const u64 g = ceil_div(items, per);
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

// One round or level's lengths: known to the host (read back) or not.
struct Known {
    bool yes;
    u32 v;
};

struct RoundCtx {
    const SortJob &J;
    SortWs &w;
    u64 n;  // strings of the whole sort (bounds every list)
    u32 SM, TL;
    u32 W;  // radix digit bits (8, or 11 with tiles >= 4096 and a cutover >= 512)
};

static u32 digit_bits_for(u32 SM, u32 TL) { return (g_digit_bits == 11 && TL >= 4096 && SM >= 512) ? 11u : 8u; }

static int scan_u32(RoundCtx &C, u32 *arr, const u32 *n_dev, Known k)
{
    if (k.yes) return ss_scan_exclusive<u32>(arr, arr, k.v, (u32 *)C.w.scan_scratch, C.J.stream);
    return ss_scan_exclusive_dev<u32>(arr, arr, n_dev, 1, C.w.dscan, C.J.stream);
}

// The part of a round before the radix levels: skip, keys, routing.
static int round_head(RoundCtx &C, Known nact, Known atiles, u64 round_elems, bool first = false)
{
    SortWs &w = C.w;
    const SortJob &J = C.J;
    hipStream_t st = J.stream;
    const u64 n = C.n;
    k_round_begin<<<1, 64, 0, st>>>(w.ctr, w.hdr);
    SS_CHECK_LAUNCH();
    const u32 *nactp = w.hdr + H_ACT;
    k_round_tiles<<<grid_of(nact.yes ? nact.v : n / 2, 256, 1024), 256, 0, st>>>(w.act, nactp, ETILE, w.tstart,
                                                                               w.skipv);
    SS_CHECK_LAUNCH();
    SS_TRY(scan_u32(C, w.tstart, nactp, nact));
    const unsigned tg = atiles.yes ? grid_of(atiles.v, 1, 1u << 30) : 0u;  // (one tile per workgroup)
    {
        // algorithmic bytes: perm + offsets + one word per string, its mismatch
        // record out, plus the common prefix (added once the skips are known)
        // (seeded: the records in, the strings of members the seed left open)
        const bool sd = first && atiles.yes && J.seed_pos;
        SS_PROF("k_skip", st, (double)round_elems * (sd ? 8.0 : 44.0));
        if (sd) k_skip<false, true><<<tg, NT, 0, st>>>(w.act, w.tstart, nactp, J.bytes, J.N, J.off, J.vals, w.skipv, J.seed_word, J.seed_pos, J.seed_ok);
        // (tiles of small segments, as later rounds leave them, hold few
        // members: one wavefront per tile then keeps four times as many in
        // flight)
        else if (atiles.yes && round_elems < 64ull * atiles.v)
            k_skip<false, false, 64><<<tg, 64, 0, st>>>(w.act, w.tstart, nactp, J.bytes, J.N, J.off, J.vals, w.skipv, w.mword, w.mpr);
        else if (atiles.yes) k_skip<false><<<tg, NT, 0, st>>>(w.act, w.tstart, nactp, J.bytes, J.N, J.off, J.vals, w.skipv, w.mword, w.mpr);
        else k_skip<true><<<grid_of(n, ETILE, resident(k_skip<true>, NT)), NT, 0, st>>>(w.act, w.tstart, nactp, J.bytes, J.N, J.off, J.vals, w.skipv, w.mword, w.mpr);
    }
    SS_CHECK_LAUNCH();
    {
        // the first round of a seeded sort keeps its records in the seed
        const bool sd = first && atiles.yes && J.seed_pos;
        u64 *mw = sd ? J.seed_word : w.mword;
        uint2 *mp = sd ? J.seed_pos : w.mpr;
        SS_PROF("k_keys", st, (double)round_elems * 24.0);  // mismatch record in, key out
        if (atiles.yes && round_elems < 64ull * atiles.v)  // (small tiles: one wavefront each, as in the skip)
            k_keys<false, 64><<<tg, 64, 0, st>>>(w.act, w.tstart, nactp, J.bytes, J.N, J.off, J.vals, w.skipv, mw, mp, w.keyA);
        else if (atiles.yes) k_keys<false><<<tg, NT, 0, st>>>(w.act, w.tstart, nactp, J.bytes, J.N, J.off, J.vals, w.skipv, mw, mp, w.keyA);
        else k_keys<true><<<grid_of(n, ETILE, resident(k_keys<true>, NT)), NT, 0, st>>>(w.act, w.tstart, nactp, J.bytes, J.N, J.off, J.vals, w.skipv, mw, mp, w.keyA);
    }
    SS_CHECK_LAUNCH();
    k_classify<<<grid_of(nact.yes ? nact.v : n / 2, 256, 1024), 256, 0, st>>>(w.act, nactp, w.skipv, C.SM, C.TL,
                                                                             w.tiny, w.small, w.largeA, w.ctr);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

// One radix level over the list LA (its length in ctr[C_LARGE] when the level
// starts); its sub-lists go to LB and the round's lists.
template <u32 W>
static int radix_level_w(RoundCtx &C, Seg *LA, Seg *LB, Known nlarge, Known ltiles, u64 lelem)
{
    constexpr u32 NB = Digits<W>::NB;
    SortWs &w = C.w;
    const SortJob &J = C.J;
    hipStream_t st = J.stream;
    const u64 n = C.n;
    k_level_begin<<<1, 64, 0, st>>>(w.ctr, w.hdr, NB);
    SS_CHECK_LAUNCH();
    const u32 *nlp = w.hdr + H_LARGE;
    k_level_tiles<<<grid_of(nlarge.yes ? nlarge.v : n / 128, 256, 1024), 256, 0, st>>>(LA, nlp, C.TL, w.tstart,
                                                                                     w.smin, w.smax);
    SS_CHECK_LAUNCH();
    SS_TRY(scan_u32(C, w.tstart, nlp, nlarge));
    const unsigned tg = ltiles.yes ? grid_of(ltiles.v, 1, 1u << 30) : 0u;  // (one tile per workgroup)
    {
        SS_PROF("k_hist", st, (double)lelem * 8.0);  // read the keys
        if (ltiles.yes) k_hist<false, W><<<tg, NT, 0, st>>>(LA, w.tstart, nlp, C.TL, w.keyA, w.keyB, w.hist, w.smin, w.smax);
        else k_hist<true, W><<<grid_of(n, C.TL, resident(k_hist<true, W>, NT)), NT, 0, st>>>(LA, w.tstart, nlp, C.TL, w.keyA, w.keyB, w.hist, w.smin, w.smax);
    }
    SS_CHECK_LAUNCH();
    if (ltiles.yes) SS_TRY(ss_scan_exclusive<u32>(w.hist, w.hist, (u64)ltiles.v * NB, (u32 *)w.scan_scratch, st));
    else SS_TRY(ss_scan_exclusive_dev<u32>(w.hist, w.hist, w.hdr + H_HIST, 1, w.dscan, st));
    EmitOut eo{w.tiny, w.small, LB, w.nxt, w.ident, w.bnd, w.ctr, w.scat, w.kinds, C.SM, C.TL};
    constexpr u32 SPG = EPB / Digits<W>::DPT;
    if (nlarge.yes) k_emit<false, W><<<grid_of(nlarge.v, SPG, 1u << 30), 256, 0, st>>>(LA, w.tstart, nlp, w.hist, w.smin, w.smax, eo);
    else k_emit<true, W><<<grid_of(n / 128, SPG, resident(k_emit<true, W>, 256)), 256, 0, st>>>(LA, w.tstart, nlp, w.hist, w.smin, w.smax, eo);
    SS_CHECK_LAUNCH();
    {
        SS_PROF("k_scatter", st, (double)lelem * 24.0);  // key+payload in and out
        if (ltiles.yes) k_scatter<false, W><<<tg, NT, 0, st>>>(LA, w.tstart, nlp, C.TL, w.hist, w.scat, w.keyA, J.vals, w.keyB, w.valB);
        else k_scatter<true, W><<<grid_of(n, C.TL, resident(k_scatter<true, W>, NT)), NT, 0, st>>>(LA, w.tstart, nlp, C.TL, w.hist, w.scat, w.keyA, J.vals, w.keyB, w.valB);
    }
    SS_CHECK_LAUNCH();
    {
        SS_PROF("k_settle", st, (double)lelem * 8.0);  // at most the scattered keys read back
        if (ltiles.yes) k_settle<false, W><<<tg, NT, 0, st>>>(LA, w.tstart, nlp, C.TL, w.scat, w.kinds, w.keyB, w.valB, w.keyA, J.vals);
        else k_settle<true, W><<<grid_of(n, C.TL, resident(k_settle<true, W>, NT)), NT, 0, st>>>(LA, w.tstart, nlp, C.TL, w.scat, w.kinds, w.keyB, w.valB, w.keyA, J.vals);
    }
    SS_CHECK_LAUNCH();
    return SS_OK;
}

static int radix_level(RoundCtx &C, Seg *LA, Seg *LB, Known nlarge, Known ltiles, u64 lelem)
{
    return C.W == 11 ? radix_level_w<11>(C, LA, LB, nlarge, ltiles, lelem)
                     : radix_level_w<8>(C, LA, LB, nlarge, ltiles, lelem);
}

// The part of a round after the radix levels: small sorts, boundary LCPs,
// equal strings.  h (when known) holds the counters after the last level.
static int round_tail(RoundCtx &C, const u32 *h)
{
    SortWs &w = C.w;
    const SortJob &J = C.J;
    hipStream_t st = J.stream;
    const u64 n = C.n;
    u32 *lcp = J.lcp;
    const bool known = h != nullptr;
    if (!known || h[C_TINY] > 0) {
        SS_PROF("k_wave_sort", st, known ? (double)h[C_TINYN] * 28.0 : 0.0);  // key+payload in/out, LCP out
        if (known)
            k_wave_sort<false><<<grid_of(h[C_TINY], WS_SPB, 1u << 30), 256, 0, st>>>(
                w.tiny, w.ctr + C_TINY, w.keyA, J.vals, w.keyB, w.valB, lcp, w.nxt, w.ctr, J.bytes, J.N, J.off);
        else
            k_wave_sort<true><<<grid_of(n / 2, WS_SPB, resident(k_wave_sort<true>, 256)), 256, 0, st>>>(
                w.tiny, w.ctr + C_TINY, w.keyA, J.vals, w.keyB, w.valB, lcp, w.nxt, w.ctr, J.bytes, J.N, J.off);
        SS_CHECK_LAUNCH();
    }
    if (!known || h[C_SMALL] > 0) {
        k_sizes<<<grid_of(known ? h[C_SMALL] : n / 2, 256, 1024), 256, 0, st>>>(w.small, w.ctr + C_SMALL, w.spref);
        SS_CHECK_LAUNCH();
        SS_TRY(scan_u32(C, w.spref, w.ctr + C_SMALL, Known{known, known ? h[C_SMALL] : 0u}));
        SS_PROF("k_lds_sort", st, known ? (double)h[C_SMALLN] * 28.0 : 0.0);  // key+payload in/out, LCP out
        if (known)
            k_lds_sort<false><<<grid_of(h[C_SMALLN], C.SM, 1u << 30), LDS_NT, 0, st>>>(
                w.small, w.spref, w.ctr + C_SMALL, C.SM, w.keyA, J.vals, w.keyB, w.valB, lcp, w.nxt, w.ctr);
        else
            k_lds_sort<true><<<grid_of(n, C.SM, resident(k_lds_sort<true>, LDS_NT)), LDS_NT, 0, st>>>(
                w.small, w.spref, w.ctr + C_SMALL, C.SM, w.keyA, J.vals, w.keyB, w.valB, lcp, w.nxt, w.ctr);
        SS_CHECK_LAUNCH();
    }
    if (!known || h[C_BND] > 0) {
        k_boundary<<<grid_of(known ? h[C_BND] : n, 256, 1024), 256, 0, st>>>(w.bnd, w.ctr + C_BND, w.keyA, lcp);
        SS_CHECK_LAUNCH();
    }
    if (!known || h[C_IDENT] > 0) {
        k_tile_counts<<<grid_of(known ? h[C_IDENT] : n / 2, 256, 1024), 256, 0, st>>>(w.ident, w.ctr + C_IDENT,
                                                                                    ETILE, w.tstart);
        SS_CHECK_LAUNCH();
        SS_TRY(scan_u32(C, w.tstart, w.ctr + C_IDENT, Known{known, known ? h[C_IDENT] : 0u}));
        if (known)
            k_ident<false><<<grid_of(h[C_ITILES], 1, 1u << 30), NT, 0, st>>>(w.ident, w.tstart, w.ctr + C_IDENT, lcp);
        else
            k_ident<true><<<grid_of(n, ETILE, resident(k_ident<true>, NT)), NT, 0, st>>>(w.ident, w.tstart, w.ctr + C_IDENT, lcp);
        SS_CHECK_LAUNCH();
    }
    return SS_OK;
}

// Host-driven rounds: the host reads the counters once after the routing,
// once per radix level and once at the end of a round, sizes every grid from
// them and stops when no segment is unresolved.  The caller has put the first
// round's segments in w.act and their count, tiles and strings in
// ctr[C_NEXT], ctr[C_NTILES], ctr[C_NELEM].
int sort_rounds(const SortJob &J, SortWs &w, u32 nact, u32 atiles)
{
    RoundCtx C{J, w, 0, (u32)g_small_max, (u32)g_tile, 8};
    C.n = J.n_total;
    C.W = digit_bits_for(C.SM, C.TL);
    u32 h[C_NCTR];
    u64 round_elems = J.n_first;
    bool first = true;
    while (nact > 0) {
        SS_TRY(round_head(C, Known{true, nact}, Known{true, atiles}, round_elems, first));
        SS_TRY(ss_read_u32(w.ctr, h, C_NCTR, J.stream));
        // (a seeded first round's common prefix was read by the pass that made the seed)
        if (!(first && J.seed_pos)) ss_prof_add_bytes("k_skip", (double)(h[10] | ((u64)h[11] << 32)));
        first = false;
        u32 nlarge = h[C_LARGE], ltiles = h[C_LTILES], lelem = h[C_LELEM];
        Seg *LA = w.largeA, *LB = w.largeB;
        while (nlarge > 0) {
            SS_TRY(radix_level(C, LA, LB, Known{true, nlarge}, Known{true, ltiles}, lelem));
            SS_TRY(ss_read_u32(w.ctr, h, C_NCTR, J.stream));
            nlarge = h[C_LARGE];
            ltiles = h[C_LTILES];
            lelem = h[C_LELEM];
            Seg *tmp = LA; LA = LB; LB = tmp;
        }
        SS_TRY(round_tail(C, h));
        SS_TRY(ss_read_u32(w.ctr, h, C_NCTR, J.stream));
        nact = h[C_NEXT];
        atiles = h[C_NTILES];
        round_elems = h[C_NELEM];
        Seg *tmp = w.act; w.act = w.nxt; w.nxt = tmp;
    }
    return SS_OK;
}

// Device-driven rounds: `rounds` rounds of as many levels as a key has digits
// are enqueued with fixed grids and nothing is read back (the launch sequence
// can be captured in a graph); rounds and levels without work find empty
// lists.  hdr[H_REMAIN] receives the number of segments still unresolved
// afterwards (0: the sort is complete).
__global__ void k_remaining(const u32 *ctr, u32 *hdr, u32 *status)
{
    hdr[H_REMAIN] = ctr[C_NEXT];
    if (status) *status = ctr[C_NEXT];
}

// The next round's segments back into the first list (after an odd number of
// rounds they are in the second), so that a continuation finds them there.
__global__ void k_copy_segs(const Seg *src, const u32 *cnt, Seg *dst)
{
    const u32 c = *cnt;
    GSTRIDE(j, c) dst[j] = src[j];
}

static int sort_rounds_device(const SortJob &J, SortWs &w, u32 rounds, u32 *status)
{
    Seg *const act0 = w.act;
    RoundCtx C{J, w, J.n_total, (u32)g_small_max, (u32)g_tile, 8};
    C.W = digit_bits_for(C.SM, C.TL);
    const u32 levels = C.W == 11 ? Digits<11>::LEVELS : Digits<8>::LEVELS;
    const Known unknown{false, 0};
    for (u32 r = 0; r < rounds; r++) {
        SS_TRY(round_head(C, unknown, unknown, 0));
        Seg *LA = w.largeA, *LB = w.largeB;
        for (u32 l = 0; l < levels; l++) {
            SS_TRY(radix_level(C, LA, LB, unknown, unknown, 0));
            Seg *tmp = LA; LA = LB; LB = tmp;
        }
        SS_TRY(round_tail(C, nullptr));
        Seg *tmp = w.act; w.act = w.nxt; w.nxt = tmp;
    }
    k_remaining<<<1, 1, 0, J.stream>>>(w.ctr, w.hdr, status);
    SS_CHECK_LAUNCH();
    if (w.act != act0) {
        k_copy_segs<<<grid_of(J.n_total / 2, 256, 1024), 256, 0, J.stream>>>(w.act, w.ctr + C_NEXT, act0);
        SS_CHECK_LAUNCH();
    }
    return SS_OK;
}

// ------------------------------------------------------------ entry points

__global__ void k_iota(u32 *p, u32 n)
{
    u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

__global__ void k_zero_u32(u32 *p, u32 count)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// The whole array as the first round's one segment (n >= 2), with its counts.
__global__ void k_init_single(Seg *act, u32 n, u32 *lcp, u32 *ctr)
{
    act[0] = Seg{0, n, 0, SEG_SKIP};
    lcp[0] = 0;
    for (u32 j = 0; j < C_NCTR; j++) ctr[j] = 0;
    ctr[C_NEXT] = 1;
    ctr[C_NTILES] = (n + ETILE - 1) / ETILE;
    ctr[C_NELEM] = n;
}

// One segment per set of two or more strings (the counters are zero before).
// A set whose bounds are not well placed (set_off non-decreasing from 0 to n)
// raises ctr[C_BADSET] and writes nothing, so a malformed set_off never leads
// outside the arrays.
__global__ void k_init_sets(const u64 *set_off, u32 nsets, u64 n, Seg *act, u32 *ctr, u32 *lcp)
{
    u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = j < nsets;
    u32 b = 0, e = 0;
    if (valid) {
        const u64 b64 = set_off[j], e64 = set_off[j + 1];
        if (e64 < b64 || e64 > n || (j == 0 && b64 != 0) || (j + 1 == nsets && e64 != n)) {
            atomicOr(&ctr[C_BADSET], 1u);
            valid = false;
        } else {
            b = (u32)b64;
            e = (u32)e64;
            if (e > b) lcp[b] = 0;
        }
    }
    bool two = valid && e > b + 1;
    u32 a = wave_append(two, &ctr[C_NEXT]);
    if (two) act[a] = Seg{b, e, 0, SEG_SKIP};
    wave_add(two ? (e - b + ETILE - 1) / ETILE : 0u, &ctr[C_NTILES]);
    wave_add(two ? e - b : 0u, &ctr[C_NELEM]);
}

// A malformed set_off found by k_init_sets leaves no segment to sort: every
// set's work is dropped (nothing is written beyond the initial identity).
__global__ void k_drop_if_bad(u32 *ctr, u32 *status)
{
    if (ctr[C_BADSET]) {
        ctr[C_NEXT] = 0;
        ctr[C_NTILES] = 0;
        ctr[C_NELEM] = 0;
    }
    if (status) status[1] = ctr[C_BADSET] ? 1u : 0u;
}

// Input indices within each set instead of the whole array, once the sort is
// complete (*remaining == 0; a sort left incomplete keeps global indices, as
// its continuation needs them).
__global__ void k_localize(const u64 *set_off, u32 nsets, u32 n, u32 *perm, const u32 *remaining)
{
    u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (remaining && *remaining)) return;
    // largest j with set_off[j] <= i
    u32 lo = 0, hi = nsets;
    while (hi - lo > 1) {
        u32 mid = (lo + hi) >> 1;
        if (set_off[mid] <= i) lo = mid;
        else hi = mid;
    }
    perm[i] -= (u32)set_off[lo];
}

extern "C" size_t ss_sort_workspace(uint64_t n)
{
    WsCounter c;
    SortWs w;
    sort_ws_layout(n, &w, nullptr, &c);
    return c.used;
}

static int sort_common_checks(const uint8_t *bytes, const uint64_t *offsets, uint64_t n, uint32_t *perm)
{
    if (n >= 0xFFFFFFFFull) {
        ss_set_error("n = %llu exceeds the 32-bit index limit", (unsigned long long)n);
        return SS_ERR_TOO_LARGE;
    }
    if (n > 0 && (!offsets || !perm)) {
        ss_set_error("null offsets or perm");
        return SS_ERR_INVALID_ARG;
    }
    (void)bytes;
    return SS_OK;
}

// Few strings (n <= RANK_MAX): one launch, no rounds.  Block i ranks string i
// among all others, (string, index) order: rank = #{ j : s_j < s_i, or s_j =
// s_i and j < i }.  The LCP with the predecessor in sorted order is the largest
// LCP of s_i with any string ranked before it (LCPs along a sorted sequence
// are range minima of the adjacent ones).
#define RANK_MAX 256
#define RANK_NT 512
__global__ __launch_bounds__(RANK_NT) void k_rank_sort(const u8 *bytes, u64 N, const u64 *off, u32 n, u32 *perm,
                                                       u32 *lcp)
{
    __shared__ u32 s_cnt[RANK_NT / 64], s_max[RANK_NT / 64];
    const u32 i = blockIdx.x;
    const u32 wv = threadIdx.x >> 6;
    const u64 oi = off[i], li = off[i + 1] - oi;
    u32 cnt = 0, mx = 0;
    for (u32 j = wv; j < n; j += RANK_NT / 64) {
        if (j == i) continue;  // uniform over the wavefront
        const u64 oj = off[j], lj = off[j + 1] - oj;
        u64 l;
        const int c = wave_str_cmp(bytes, N, oj, lj, oi, li, &l);
        if (c < 0 || (c == 0 && j < i)) {
            cnt++;
            if (l > mx) mx = (u32)l;
        }
    }
    if ((threadIdx.x & 63) == 0) { s_cnt[wv] = cnt; s_max[wv] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 r = 0, m = 0;
        for (u32 w = 0; w < RANK_NT / 64; w++) { r += s_cnt[w]; m = s_max[w] > m ? s_max[w] : m; }
        perm[r] = i;
        if (lcp) lcp[r] = m;
    }
}

// The first-round seed's arrays (layout: 256-byte header whose word 0 says
// whether the seed was written, the mismatch words (n), the records (n)).
static void attach_seed(SortJob &J, void *seed, u64 n)
{
    J.seed_ok = (const u32 *)seed;
    J.seed_word = (u64 *)((u8 *)seed + 256);
    J.seed_pos = (uint2 *)((u8 *)seed + 256 + 8 * n);
}

static int sort_single(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n, void *seed,
                       uint32_t *perm, uint32_t *lcp, void *ws, size_t ws_bytes, void *stream)
{
    SS_TRY(sort_common_checks(bytes, offsets, n, perm));
    if (n == 0) return SS_OK;
    hipStream_t st = (hipStream_t)stream;
    WsArena a(ws, ws_bytes);
    SortWs w;
    sort_ws_layout(n, &w, &a, nullptr);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_sort_workspace(n));
        return SS_ERR_WORKSPACE;
    }
    if (n <= RANK_MAX) {
        k_rank_sort<<<(unsigned)n, RANK_NT, 0, st>>>(bytes, N, offsets, (u32)n, perm, lcp);
        SS_CHECK_LAUNCH();
        return SS_OK;
    }
    SortJob J{bytes, N, offsets, perm, lcp ? lcp : w.lcp_scratch, st, n, n};
    if (seed) attach_seed(J, seed, n);
    k_iota<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(perm, (u32)n);
    SS_CHECK_LAUNCH();
    k_init_single<<<1, 1, 0, st>>>(w.act, (u32)n, J.lcp, w.ctr);
    SS_CHECK_LAUNCH();
    return sort_rounds(J, w, 1, (u32)ceil_div(n, ETILE));
}

extern "C" int ss_sort(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                       uint32_t *perm, uint32_t *lcp, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    return sort_single(bytes, N, offsets, n, nullptr, perm, lcp, ws, ws_bytes, stream);
}

extern "C" int ss_sort_seeded(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                              void *sort_seed, uint32_t *perm, uint32_t *lcp, void *ws, size_t ws_bytes,
                              void *stream)
{
    ss_clear_error();
    if (!sort_seed) {
        ss_set_error("null sort_seed");
        return SS_ERR_INVALID_ARG;
    }
    return sort_single(bytes, N, offsets, n, sort_seed, perm, lcp, ws, ws_bytes, stream);
}

// The checks and first-round set-up shared by both batch forms.
static int batch_setup(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                       const uint64_t *set_off, uint32_t num_sets, uint32_t *perm, uint32_t *lcp, uint32_t flags,
                       void *ws, size_t ws_bytes, hipStream_t st, SortWs &w, SortJob &J)
{
    SS_TRY(sort_common_checks(bytes, offsets, n, perm));
    if (num_sets == 0 || !set_off) {
        ss_set_error("batch needs num_sets >= 1 and set_off");
        return SS_ERR_INVALID_ARG;
    }
    if (flags & ~(SS_BATCH_GLOBAL_IDS | SS_BATCH_CONTINUE)) {
        ss_set_error("unknown flags 0x%x", flags);
        return SS_ERR_INVALID_ARG;
    }
    if (n == 0) return SS_OK;
    WsArena a(ws, ws_bytes);
    sort_ws_layout(n, &w, &a, nullptr);
    if (a.overflow || !ws) {
        ss_set_error("workspace too small: need %zu bytes", ss_sort_workspace(n));
        return SS_ERR_WORKSPACE;
    }
    J = SortJob{bytes, N, offsets, perm, lcp ? lcp : w.lcp_scratch, st, 0, n};
    if (flags & SS_BATCH_CONTINUE) return SS_OK;  // the state of an incomplete device-driven sort
    k_iota<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(perm, (u32)n);
    SS_CHECK_LAUNCH();
    k_zero_u32<<<1, 64, 0, st>>>(w.ctr, C_NCTR);
    SS_CHECK_LAUNCH();
    k_init_sets<<<(unsigned)ceil_div(num_sets, 256), 256, 0, st>>>(set_off, num_sets, n, w.act, w.ctr, J.lcp);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

static int sort_batch_impl(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                           const uint64_t *set_off, uint32_t num_sets, void *seed, uint32_t *perm_local,
                           uint32_t *lcp, uint32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    SortWs w;
    SortJob J{};
    SS_TRY(batch_setup(bytes, N, offsets, n, set_off, num_sets, perm_local, lcp, flags, ws, ws_bytes, st, w, J));
    if (n == 0) return SS_OK;
    if (seed) attach_seed(J, seed, n);
    u32 h[C_NCTR];
    SS_TRY(ss_read_u32(w.ctr, h, C_NCTR, st));
    if (h[C_BADSET]) {
        ss_set_error("set_off must be non-decreasing with set_off[0] = 0 and set_off[num_sets] = n");
        return SS_ERR_INVALID_ARG;
    }
    J.n_first = h[C_NELEM];
    SS_TRY(sort_rounds(J, w, h[C_NEXT], h[C_NTILES]));
    if (!(flags & SS_BATCH_GLOBAL_IDS)) {
        k_localize<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(set_off, num_sets, (u32)n, perm_local, nullptr);
        SS_CHECK_LAUNCH();
    }
    return SS_OK;
}

extern "C" int ss_sort_batch(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                             const uint64_t *set_off, uint32_t num_sets, uint32_t *perm_local,
                             uint32_t *lcp, uint32_t flags, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    return sort_batch_impl(bytes, N, offsets, n, set_off, num_sets, nullptr, perm_local, lcp, flags, ws, ws_bytes,
                           stream);
}

extern "C" int ss_sort_batch_seeded(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                    const uint64_t *set_off, uint32_t num_sets, void *sort_seed,
                                    uint32_t *perm_local, uint32_t *lcp, uint32_t flags, void *ws,
                                    size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (!sort_seed || (flags & SS_BATCH_CONTINUE)) {
        ss_set_error(!sort_seed ? "null sort_seed" : "a seeded sort cannot continue a device-driven one");
        return SS_ERR_INVALID_ARG;
    }
    return sort_batch_impl(bytes, N, offsets, n, set_off, num_sets, sort_seed, perm_local, lcp, flags, ws,
                           ws_bytes, stream);
}

extern "C" uint32_t ss_sort_batch_device_rounds(uint32_t max_len)
{
    // a round consumes at least 7 bytes of every string it keeps
    return max_len / 7 + 2;
}

extern "C" int ss_sort_batch_device(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                                    const uint64_t *set_off, uint32_t num_sets, uint32_t *perm_local,
                                    uint32_t *lcp, uint32_t flags, uint32_t rounds, uint32_t *status, void *ws,
                                    size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (!status) {
        ss_set_error("status is required");
        return SS_ERR_INVALID_ARG;
    }
    if (rounds == 0 || rounds > 1024) {
        ss_set_error("rounds must be 1..1024");
        return SS_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    SortWs w;
    SortJob J{};
    SS_TRY(batch_setup(bytes, N, offsets, n, set_off, num_sets, perm_local, lcp, flags, ws, ws_bytes, st, w, J));
    if (n == 0) {
        k_zero_u32<<<1, 64, 0, st>>>(status, 2);
        SS_CHECK_LAUNCH();
        return SS_OK;
    }
    if (!(flags & SS_BATCH_CONTINUE)) {
        k_drop_if_bad<<<1, 1, 0, st>>>(w.ctr, status);
        SS_CHECK_LAUNCH();
    }
    SS_TRY(sort_rounds_device(J, w, rounds, status));
    if (!(flags & SS_BATCH_GLOBAL_IDS)) {
        k_localize<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(set_off, num_sets, (u32)n, perm_local,
                                                               w.ctr + C_NEXT);
        SS_CHECK_LAUNCH();
    }
    return SS_OK;
}
