// Segmented string sort machinery (workspace layout and the round driver).
#pragma once
#include "common.hpp"

// A contiguous range [begin, end) of sorted positions whose strings share a
// known prefix of `depth` bytes.  aux: bits 0..3 = current key byte of a radix
// pass, bit 4 = compute the common-prefix skip first, bit 5 = the segment's
// keys and payload are in the B arrays (radix levels alternate between A and
// B; everything final is in A).
struct Seg {
    u32 begin, end, depth, aux;
};
enum { SEG_SKIP = 16, SEG_INB = 32 };

struct SortWs {
    u64 *keyA, *keyB, *mword;  // mword, mpr: each member's first mismatch with its segment's first string
    uint2 *mpr;
    u32 *valB, *lcp_scratch;
    Seg *act, *nxt, *tiny, *small, *ident, *largeA, *largeB;
    uint2 *bnd;
    u32 *skipv;
    u64 *smin, *smax;
    u8 *scat;
    u8 *kinds;  // per radix segment and digit: what the bucket became
    u32 *tstart, *spref, *hist;
    u64 *scan_scratch;
    u32 *dscan;  // scratch of the device-length scans
    u32 *ctr;
    u32 *hdr;    // list lengths of the current round and level (device)
};

struct SortJob {
    const u8 *bytes;
    u64 N;
    const u64 *off;
    u32 *vals;  // payload: input indices
    u32 *lcp;   // LCP output
    hipStream_t stream;
    u64 n_first;  // strings in the first round's segments (for byte accounting)
    u64 n_total;  // strings of the whole sort (bounds every list)
    // First-round seed (null: none): the mismatch records of the first
    // round's one segment, used in place of the workspace's when *seed_ok.
    u64 *seed_word;
    uint2 *seed_pos;
    const u32 *seed_ok;
};

void sort_ws_layout(u64 n, SortWs *w, WsArena *a, WsCounter *c);
// Host-driven rounds from nact segments in w.act covering `atiles` element
// tiles of 2048 (their count, tiles and strings also in the counters).
int sort_rounds(const SortJob &J, SortWs &w, u32 nact, u32 atiles);
