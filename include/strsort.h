/*
 * strsort -- one GPU's share of the data-parallel hot path of distributed
 * string sorting, for AMD Instinct MI355X (gfx950).
 *
 * Method: "Scalable Distributed String Sorting" (Kurpicz, Mehnert, Sanders,
 * Schimek).  The entry points below are the local steps each processing
 * element runs: sort + LCP array (Section 3, "Initialization"), exact and
 * approximate distinguishing prefixes (Section 2; Section 4 with Appendix B
 * and C), bucket computation and LCP compression (Section 3, steps 1-2;
 * Section 2, "Algorithmic Building Blocks"), and LCP-aware merging of sorted
 * runs (Section 3, step 3).  The message exchange between processing elements
 * is replaced by runs already resident in device memory.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A string array is (bytes, N, offsets, n): string i occupies
 *   bytes[offsets[i] .. offsets[i+1]), offsets has n+1 non-decreasing entries
 *   and offsets[n] <= N.  Strings are unsigned byte sequences with explicit
 *   lengths; a proper prefix sorts before its extensions (the end-of-string
 *   sentinel of Section 2 sorts below every byte, 0x00 included).
 * - Order arrays (perm, lcp, front-coded arrays) are indexed by sorted
 *   position; per-string properties (dist) are indexed by input index.
 * - Equal strings are ordered by input index (the sort is stable).
 * - lcp[0] = 0 and lcp[i] = number of equal leading bytes of the strings at
 *   sorted positions i-1 and i.
 * - Every pointer is DEVICE memory owned by the caller unless its comment says
 *   "host".  The library allocates no device memory: scratch comes from the
 *   caller's workspace `ws` of `ws_bytes` bytes, sized by the matching
 *   *_workspace() query.  `stream` is a hipStream_t (NULL = default stream).
 * - Calls are enqueued on `stream`.  Calls that iterate (sort rounds, doubling
 *   rounds, merge levels) read small counters back to the host and therefore
 *   synchronise `stream` between iterations; outputs are complete when the call
 *   returns.  Concurrent calls on different streams with different workspaces
 *   are independent.
 * - Return value: SS_OK or a negative SS_ERR_* code; ss_last_error() gives a
 *   thread-local message.  No call aborts or throws across this boundary.
 * - Limits: n < 2^32 - 1; every string shorter than 2^32 - 1 bytes.
 */
#ifndef STRSORT_H
#define STRSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SS_OK 0
#define SS_ERR_INVALID_ARG (-1)  /* null pointer, bad size, bad parameter      */
#define SS_ERR_WORKSPACE (-2)    /* ws_bytes smaller than the *_workspace query */
#define SS_ERR_TOO_LARGE (-3)    /* n or a length beyond the 32-bit limits     */
#define SS_ERR_HIP (-4)          /* a HIP runtime call failed (text in last_error) */
#define SS_ERR_CAPACITY (-5)     /* an output buffer is smaller than needed    */

/* Thread-local text of the last error (empty if none).  Host string. */
const char *ss_last_error(void);

/* Library version (major*100 + minor). */
int ss_version(void);

/* ------------------------------------------------------------------ sort */

/* Workspace bytes for ss_sort / ss_sort_batch on n strings. */
size_t ss_sort_workspace(uint64_t n);

/* Sort + LCP array (Section 3, "Initialization": sort the local string array;
 * the LCP array is obtained as a by-product).
 *   perm[i] (out, n)  input index of the i-th smallest string (stable).
 *   lcp[i]  (out, n)  LCP array of the sorted order; may be NULL.
 * Errors: INVALID_ARG (null bytes/offsets/perm with n > 0), TOO_LARGE,
 * WORKSPACE, HIP. */
int ss_sort(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
            uint32_t *perm, uint32_t *lcp, void *ws, size_t ws_bytes, void *stream);

/* ss_sort with its first round's comparisons against the first string taken
 * from sort_seed, written by ss_dist_prefix_first_seed on the same strings
 * (on a stream ordered after that call).  Same results as ss_sort.  The sort
 * overwrites the seed's records (they become its first round's).  A seed
 * whose header says it was not written is ignored; a seed of other strings
 * gives wrong results.  Errors as ss_sort, INVALID_ARG for a null
 * sort_seed. */
int ss_sort_seeded(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n, void *sort_seed,
                   uint32_t *perm, uint32_t *lcp, void *ws, size_t ws_bytes, void *stream);
/* ss_sort_batch with the first round taken from a seed that
 * ss_dist_prefix_first_seed wrote for the same strings and the same set_off.
 * Same results as ss_sort_batch; INVALID_ARG also for a null sort_seed or
 * SS_BATCH_CONTINUE. */
int ss_sort_batch_seeded(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                         const uint64_t *set_off, uint32_t num_sets, void *sort_seed, uint32_t *perm,
                         uint32_t *lcp, uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* Many independent sorts in one launch sequence (one sort per set, as each
 * processing element sorts its own array in Section 3).  set_off (device,
 * num_sets+1 entries, non-decreasing, set_off[0] = 0, set_off[num_sets] = n)
 * gives the string-index bounds of each set within one string array.
 *   perm[i] (out, n)  the string at position i of its set's sorted order
 *                     (positions are global): its index WITHIN the set, or,
 *                     with SS_BATCH_GLOBAL_IDS in flags, its index in the
 *                     whole string array.
 *   lcp[i] (out, n)   LCP array of each set (0 at each set start); may be NULL.
 * Uses the ss_sort workspace for n.  INVALID_ARG if set_off is malformed
 * (checked on the device; the call reads one word back) or flags has an
 * unknown bit. */
#define SS_BATCH_GLOBAL_IDS 1u
/* Continue a device-driven batch sort that ended with unresolved segments
 * (ss_sort_batch_device's status[0] > 0): same arguments and workspace as that
 * call, whose state (the order so far and the segments left) the workspace
 * holds; ss_sort_batch finishes it host-driven, ss_sort_batch_device runs
 * `rounds` more rounds.  Indices become set-local (without
 * SS_BATCH_GLOBAL_IDS) only once the sort is complete. */
#define SS_BATCH_CONTINUE 2u
int ss_sort_batch(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                  const uint64_t *set_off, uint32_t num_sets, uint32_t *perm, uint32_t *lcp,
                  uint32_t flags, void *ws, size_t ws_bytes, void *stream);

/* The batched sort with the rounds driven from the device, for capture in a
 * graph (ss_graph_begin / ss_graph_end) and for callers that must not wait on
 * the host: the same result as ss_sort_batch, with nothing read back and
 * nothing allocated; every launch has a fixed shape.  `rounds` sort rounds
 * (each of up to 8 radix levels) are enqueued; a round resolves at least 7
 * more bytes of every string it keeps, so ss_sort_batch_device_rounds(L)
 * rounds finish any input whose strings are at most L bytes long.
 *   status (device, 2 words, out): status[0] = segments still unresolved
 *   after the last round (0: perm and lcp are complete; else they are not,
 *   and a call with SS_BATCH_CONTINUE finishes the sort from the workspace's
 *   state), status[1] = 1 if set_off is malformed (then nothing is sorted).
 * Other arguments, outputs and workspace as in ss_sort_batch.  Rounds without
 * work cost only launches that find empty lists. */
uint32_t ss_sort_batch_device_rounds(uint32_t max_len);
int ss_sort_batch_device(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                         const uint64_t *set_off, uint32_t num_sets, uint32_t *perm, uint32_t *lcp,
                         uint32_t flags, uint32_t rounds, uint32_t *status, void *ws, size_t ws_bytes,
                         void *stream);

/* ------------------------------------------------------- LCP and dist */

/* LCP array of a given order (Section 2): lcp[0] = 0,
 * lcp[i] = lcp(s_perm[i-1], s_perm[i]).  perm (in, n), lcp (out, n); the
 * values of perm index the string array (which may hold more than n strings). */
int ss_lcp(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
           const uint32_t *perm, uint32_t *lcp, void *stream);

/* LCPs across group boundaries of a multi-group merge (Section 3: the merged
 * buckets, concatenated in bucket order, form the sorted output).  The groups
 * and runs are those given to ss_lcp_merge (run_begin, run_end: k entries;
 * group_off: groups+1 entries; all device), order = its out_id (n_out), lcp =
 * its out_lcp (in/out, n_out).  For every non-empty group g >= 1 whose first
 * output position G is > 0: lcp[G] = lcp(s_order[G-1], s_order[G]); nothing
 * else changes.  The values of order index the string array. */
int ss_join_group_lcps(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, const uint32_t *order,
                       uint64_t n_out, uint32_t k, const uint64_t *run_begin, const uint64_t *run_end,
                       uint32_t groups, const uint32_t *group_off, uint32_t *lcp, void *stream);

/* Exact distinguishing prefix length (Section 2): the characters needed to
 * rank a string, dist(s) = min(len(s), 1 + max over t != s of lcp(s, t)),
 * evaluated from the sorted neighbours: for the string at sorted position i,
 * dist = min(len, 1 + max(lcp[i], lcp[i+1])) with lcp[n] := 0.
 *   perm, lcp (in, n; a sorted order and its LCP array), dist (out, by input
 *   index: dist[perm[i]] is written for i < n). */
int ss_dist_exact(const uint64_t *offsets, uint64_t n, const uint32_t *perm,
                  const uint32_t *lcp, uint32_t *dist, void *stream);

/* The same dist from a bound instead of the string array: for the string at
 * sorted position i, any d[i] with dist <= d[i] <= len gives
 * dist = min(d[i], 1 + max(lcp[i], lcp[i+1])) (if 1 + max <= d[i] it is <=
 * len; otherwise dist = len = d[i]).  Approximate distinguishing prefixes
 * (ss_dist_prefix) qualify, and so do the fc_len values of a merge output
 * (out_len).  perm, lcp, d (in, n), dist (out, n or more, by input index:
 * dist[perm[i]]).  perm may be NULL: then dist[i] is written, by sorted
 * position (the layout of a PE's merged output, whose strings' input indices
 * belong to other PEs), and every read and write is sequential. */
int ss_dist_exact_bounded(const uint32_t *perm, const uint32_t *lcp, const uint32_t *d, uint64_t n,
                          uint32_t *dist, void *stream);

/* ----------------------------------------------------- prefix doubling */

/* Workspace bytes for ss_dist_prefix on n strings. */
size_t ss_dist_prefix_workspace(uint64_t n);

/* Approximate distinguishing prefixes by prefix doubling (Section 4; proof
 * outline in Appendix C) with exact duplicate detection (the multiplicity of
 * each key among the active strings, as Appendix B's sort-and-scan finds it;
 * here counted in a hash table of the keys).  Round t hashes the
 * l_t-prefix of every active string, l_t = init_len * 2^t; a string finishes
 * when its key is unique among the active strings or its length is <= l_t,
 * with dist_approx = min(l_t, len).  Result: dist_approx >= dist for every
 * string, whatever the hash.
 *   init_len   positive multiple of 4 (the paper's l_init; 8 in the workloads).
 *   hash_bits  keep the low hash_bits bits of each key (8..64; 64 = full key).
 *              Smaller values force collisions for testing.
 *   dist_approx (out, n, by input index).
 *   rounds_host (host, out, nullable): number of doubling rounds run.
 * Hash: Karp-Rabin modulo 2^61-1 with base 0x0B3C4D5E6F708192 over 4-byte
 * little-endian limbs of the prefix (last limb zero-padded), followed by the
 * prefix length as a final digit: key = (C*B + m) mod p.  The paper leaves
 * the hash open; this one is incremental, so round t reads only bytes
 * [l_{t-1}, l_t). */
int ss_dist_prefix(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                   uint32_t init_len, uint32_t hash_bits, uint32_t *dist_approx,
                   uint32_t *rounds_host, void *ws, size_t ws_bytes, void *stream);
/* (Synchronises the stream: the number of active strings is read back every
 * round.) */

/* ss_dist_prefix in two calls that share the workspace, so that a caller can
 * order the first pass against other work: ss_dist_prefix_first hashes every
 * string's first bytes (all rounds up to 64 bytes, or 256 bytes when a sample
 * shows long shared prefixes; it reads the sample's count back), then
 * ss_dist_prefix_rounds (same arguments, same workspace, on a stream ordered
 * after the first call) runs the remaining rounds and the duplicate
 * detection.  Together they compute exactly what ss_dist_prefix computes.
 * INVALID_ARG from ss_dist_prefix_rounds if the workspace holds no first
 * pass for init_len. */
int ss_dist_prefix_first(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                         uint32_t init_len, uint32_t hash_bits, void *ws, size_t ws_bytes, void *stream);
int ss_dist_prefix_rounds(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                          uint32_t init_len, uint32_t hash_bits, uint32_t *dist_approx,
                          uint32_t *rounds_host, void *ws, size_t ws_bytes, void *stream);

/* One read of every string's first bytes for both passes of Section 3's
 * initialization (each processing element's local sort) and Section 4's
 * prefix doubling.  The deep first pass (the one that reads 256 bytes) also
 * compares each string with the first string of its set over those bytes and
 * leaves, in sort_seed, what the sort's first round needs: the string's first
 * mismatch with that string (their LCP) and its 8 bytes there, or, for a
 * string that agrees with it over all 256 bytes, the position to go on from.
 * ss_sort_seeded / ss_sort_batch_seeded then sort without reading those
 * bytes again.
 *   set_off   (device, num_sets+1, nullable) the sets of the batch sort that
 *              will use the seed (as ss_sort_batch's); NULL: one set, for
 *              ss_sort_seeded.  The pass keeps every set's first string in
 *              LDS: with more than 16 sets it writes no seed (the seeded sort
 *              then compares everything itself).  The strings of a 32-string
 *              tile that crosses a set bound are left for the sort too.
 *   sort_seed (device, out, ss_sort_seed_bytes(n) bytes, caller-owned): a
 *              256-byte header (word 0 = 1 when the seed was written, 0 when
 *              the plain first pass ran and wrote none), then n 8-byte words
 *              and n 8-byte records.  Its contents are an implementation
 *              detail; pass it only to a seeded sort of the same strings and
 *              sets.
 *   first_pass_mode 0 = as ss_dist_prefix_first (a sample decides between the
 *              plain and the deep pass), 1 = plain, 2 = deep.
 * Otherwise exactly ss_dist_prefix_first: ss_dist_prefix_rounds continues
 * from the workspace.  Errors as ss_dist_prefix_first; INVALID_ARG for a null
 * sort_seed, a mode above 2, or set_off with num_sets = 0. */
size_t ss_sort_seed_bytes(uint64_t n);
int ss_dist_prefix_first_seed(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                              const uint64_t *set_off, uint32_t num_sets, uint32_t init_len, uint32_t hash_bits,
                              uint32_t first_pass_mode, void *sort_seed, void *ws, size_t ws_bytes, void *stream);

/* The keys of the first `rounds` prefix-doubling rounds of every string, as
 * ss_dist_prefix's rounds compute them (Section 4: round t hashes the
 * l_t-prefix, l_t = init_len * 2^t), with every string kept active:
 *   keys[t*n + i] (out, rounds*n) = key of s_i[0, min(l_t, len)), masked to
 *   hash_bits (same hash and arguments as ss_dist_prefix).
 * first_pass_mode selects the form of the first pass over rounds with
 * l_t <= 64: 0 = as ss_dist_prefix decides (a sampled probe), 1 = plain (up
 * to 64 bytes), 2 = deep (also rounds 128 and 256; only when a round of
 * exactly 64 bytes exists, else plain).  Later rounds go through the round
 * kernel, two rounds per launch where ss_dist_prefix would also do so.
 * Exposed so that the hash kernels can be checked key by key.  Uses the
 * ss_dist_prefix workspace for n.  INVALID_ARG if rounds > 32 or
 * l_{rounds-1} > 2^31. */
int ss_doubling_keys(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                     uint32_t init_len, uint32_t hash_bits, uint32_t rounds, uint32_t first_pass_mode,
                     uint64_t *keys, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------- splitters, buckets, coding */

/* One-device form of regular sampling (Section 3.1: f_j = V[j|V|/r - 1]) with
 * V = the whole sorted array: splitter_ids[j-1] = perm[ceil(j*n/r) - 1] for
 * j = 1..r-1.  perm (in, n), splitter_ids (out, r-1).  n >= 1, r >= 1. */
int ss_select_splitters(uint64_t n, const uint32_t *perm, uint32_t r, uint32_t *splitter_ids,
                        void *stream);

/* Workspace bytes for ss_select_splitters_batch (a constant). */
size_t ss_select_splitters_batch_workspace(void);

/* Regular sampling of Section 3.1 applied to every set of a batch in one
 * launch: set b is positions [set_off[b], set_off[b+1]) of perm (n_b strings),
 * and splitter_ids[b*(r-1) + j-1] = perm[set_off[b] + ceil(j*n_b/r) - 1] for
 * j = 1..r-1.  perm (in, n), set_off (in, num_sets+1), splitter_ids (out,
 * num_sets*(r-1)).  INVALID_ARG if a set is empty or set_off is not increasing
 * from 0 to n (checked on the device, so the call synchronises the stream;
 * the samples of a bad set are 0xFFFFFFFF).  ws = NULL with ws_bytes = 0:
 * no check and nothing read back (for a caller whose sets are well formed by
 * construction; a bad set's samples are still 0xFFFFFFFF, which
 * ss_gather_strings takes as empty strings). */
int ss_select_splitters_batch(const uint32_t *perm, uint64_t n, const uint64_t *set_off, uint32_t num_sets,
                              uint32_t r, uint32_t *splitter_ids, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for ss_select_splitters_chars_batch on n sorted positions. */
size_t ss_select_splitters_chars_batch_workspace(uint64_t n);

/* Character-based regular sampling (Section 3.1, "Character-Based Sampling";
 * Appendix A) of every set of a batch: samples at equally spaced positions of
 * each sorted set's character array, each shifted back to the start of the
 * string that holds it, so that buckets between them hold balanced numbers of
 * characters rather than of strings.  Set b is positions [set_off[b],
 * set_off[b+1]) of perm (values index offsets); with C_k the characters of the
 * set's first k strings and N_b = C_{n_b}, sample j (1..r-1) is at character
 * position x_j = ceil(j N_b / r) - 1 and splitter_ids[b*(r-1) + j-1] =
 * perm[set_off[b] + k] for the k with C_k <= x_j < C_{k+1} (a set without
 * characters gives its first string).  Characters are string lengths, or
 * weights[s] (device, by input index, nullable; e.g. the approximate
 * distinguishing prefixes of ss_dist_prefix, the characters prefix-doubling
 * merge sort sends).  Errors as ss_select_splitters_batch (reads one word
 * back). */
int ss_select_splitters_chars_batch(const uint32_t *perm, const uint64_t *offsets, const uint32_t *weights,
                                    uint64_t n, const uint64_t *set_off, uint32_t num_sets, uint32_t r,
                                    uint32_t *splitter_ids, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for ss_gather_strings of m strings. */
size_t ss_gather_workspace(uint64_t m);

/* Copy strings ids[0..m) of a string array into a new string array
 * (out_offsets: m+1 entries, out_offsets[0] = 0; out_bytes capacity out_cap).
 * Used to materialise splitter strings.  An id >= n is an empty string.
 * *total_host (host) receives the byte total (the call reads it back);
 * CAPACITY if out_cap is too small: out_offsets and *total_host are then
 * valid, no bytes are copied.  total_host = NULL: nothing is read back; the
 * byte total is out_offsets[m] on the device, and a string that would end
 * past out_cap is not copied (out_offsets[m] > out_cap tells the caller). */
int ss_gather_strings(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                      const uint32_t *ids, uint64_t m, uint64_t *out_offsets, uint8_t *out_bytes,
                      uint64_t out_cap, uint64_t *total_host, void *ws, size_t ws_bytes, void *stream);

/* Bucket boundaries for r-1 sorted splitters (Section 3, step 1:
 * B^j = { s : f_j < s <= f_{j+1} }, f_0 = -inf, f_r = +inf):
 * bounds[0] = 0, bounds[r] = n, bounds[j] = #{ i : s_perm[i] <= f_j }.
 * Splitters are a string array (spl_bytes, spl_N, spl_offsets, r-1 strings),
 * non-decreasing.  bounds (out, r+1). */
int ss_bucket_bounds(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                     const uint32_t *perm, const uint8_t *spl_bytes, uint64_t spl_N,
                     const uint64_t *spl_offsets, uint32_t r, uint64_t *bounds, void *stream);

/* Workspace bytes for ss_partition_encode on n strings. */
size_t ss_partition_encode_workspace(uint64_t n);

/* Split a sorted array into r buckets and LCP-compress each bucket (Section 3
 * steps 1-2 with LCP compression, Section 2; distinguishing prefixes only in
 * the prefix-doubling variant, Section 4).  Front-coded run format, per
 * sorted position i in bucket j = [run_off[j], run_off[j+1]):
 *   fc_lcp[i] = e_i = 0 at the bucket start, else lcp[i];
 *   fc_len[i] = d_i = dist[perm[i]] if dist != NULL, else the full length;
 *   fc_id[i]  = perm[i];
 *   suf[suf_off[i] .. suf_off[i+1]) = bytes s_perm[i][e_i, d_i)
 * (suf_off has n+1 entries).  Literal bytes start at suf + suf_base and every
 * suf_off entry includes suf_base, so several arrays can be encoded into one
 * shared buffer (suf_off[n] = suf_base + total literal bytes).
 * Inputs: perm, lcp (a sorted order and its LCP array), dist (by input index,
 * must satisfy dist >= min(len, lcp+1) as ss_dist_prefix guarantees; NULL =
 * full strings), splitters as in ss_bucket_bounds.  suf_cap: capacity of suf
 * in bytes (suf_base + N always suffices).  suf_total_host (host, out,
 * nullable): literal bytes written by this call.
 * Errors: CAPACITY if suf_cap is too small (fc_lcp, fc_len, fc_id, suf_off are
 * complete; no literal byte is written), INVALID_ARG if some e_i > d_i or
 * d_i > len. */
int ss_partition_encode(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                        const uint32_t *perm, const uint32_t *lcp, const uint32_t *dist,
                        const uint8_t *spl_bytes, uint64_t spl_N, const uint64_t *spl_offsets,
                        uint32_t r, uint64_t *run_off, uint32_t *fc_lcp, uint32_t *fc_len,
                        uint32_t *fc_id, uint64_t *suf_off, uint8_t *suf, uint64_t suf_base,
                        uint64_t suf_cap, uint64_t *suf_total_host, void *ws, size_t ws_bytes,
                        void *stream);

/* ss_partition_encode for num_sets sorted arrays at once (each processing
 * element splits its own array with the same splitters, Section 3 steps 1-2),
 * in one launch sequence.  Set b is the sorted positions
 * [set_off[b], set_off[b+1]) of perm/lcp (set_off: device, num_sets+1
 * entries, non-decreasing, set_off[num_sets] = n); perm values index offsets.
 * run_off (out, num_sets*(r+1)): the bucket bounds of set b, as absolute
 * positions, at run_off[b*(r+1) .. b*(r+1)+r].  The front-coded arrays cover
 * all n positions; e = 0 at every bucket start of every set.  Workspace as for
 * ss_partition_encode(n). */
int ss_partition_encode_batch(const uint8_t *bytes, uint64_t N, const uint64_t *offsets,
                              uint64_t n, const uint64_t *set_off, uint32_t num_sets,
                              const uint32_t *perm, const uint32_t *lcp, const uint32_t *dist,
                              const uint8_t *spl_bytes, uint64_t spl_N,
                              const uint64_t *spl_offsets, uint32_t r, uint64_t *run_off,
                              uint32_t *fc_lcp, uint32_t *fc_len, uint32_t *fc_id,
                              uint64_t *suf_off, uint8_t *suf, uint64_t suf_base, uint64_t suf_cap,
                              uint64_t *suf_total_host, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for ss_fc_decode on n strings. */
size_t ss_fc_decode_workspace(uint64_t n);

/* Decode k front-coded runs (format of ss_partition_encode; run_off has k+1
 * entries, device) into a string array: string i of run j is the first e_i
 * bytes of string i-1 of the same run followed by its literal bytes.
 * out_offsets (out, n+1, out_offsets[0] = 0), out_bytes (out, capacity
 * out_cap >= sum d_i, else CAPACITY). */
int ss_fc_decode(uint32_t k, const uint64_t *run_off, const uint32_t *fc_lcp,
                 const uint32_t *fc_len, const uint64_t *suf_off, const uint8_t *suf, uint64_t n,
                 uint64_t *out_offsets, uint8_t *out_bytes, uint64_t out_cap, void *ws,
                 size_t ws_bytes, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): ss_fc_decode without a
 * caller workspace and without any host read-back or allocation.  Its scratch
 * is a static device array of the library (36 MiB, one copy per GPU, held
 * until the process ends); n is limited to SS_FC_DECODE_NOALLOC_MAX entries
 * (TOO_LARGE beyond, checked before anything is enqueued).  Arguments and
 * outputs as in ss_fc_decode, except that the data-dependent checks are
 * reported on the device instead of by the return value:
 *   status (device, 1 word, out): 0 = decoded; 1 = malformed runs (nothing
 *   decoded); 2 = the decoded bytes exceed out_cap (out_offsets is complete,
 *   no byte is written).
 * The call is asynchronous on `stream` (whose device must be the current
 * device).  Every call on one GPU uses that GPU's one scratch array, which
 * keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.  The
 * first call on a device looks the array's device address up. */
#define SS_FC_DECODE_NOALLOC_MAX (1u << 22)
int ss_fc_decode_noalloc(uint32_t k, const uint64_t *run_off, const uint32_t *fc_lcp,
                         const uint32_t *fc_len, const uint64_t *suf_off, const uint8_t *suf, uint64_t n,
                         uint64_t *out_offsets, uint8_t *out_bytes, uint64_t out_cap, uint32_t *status,
                         void *stream);

/* ---------------------------------------------------------------- merge */

/* Workspace bytes for ss_lcp_merge of n_out merged strings drawn from front-
 * coded arrays of n_fc entries in k runs. */
size_t ss_lcp_merge_workspace(uint64_t n_out, uint64_t n_fc, uint32_t k);

/* LCP-aware merging of sorted front-coded runs (Section 3, step 3; the paper
 * uses an LCP loser tree, Section 2), for several independent groups of runs
 * in one call (on one device: the runs each bucket receives from every
 * processing element).
 *   Front-coded arrays (format of ss_partition_encode), n_fc entries:
 *     fc_lcp, fc_len, fc_id (n_fc), suf_off (n_fc+1), suf.  The literal of
 *     entry i is the d_i - e_i bytes at suf + suf_off[i]; suf_off[n_fc] bounds
 *     the literal buffer (arrays filled by several ss_partition_encode calls
 *     with different suf_base qualify).
 *   Runs: run j = front-coded positions [run_begin[j], run_end[j]) (device,
 *     k entries each); runs must not overlap; every non-empty run starts with
 *     e = 0 and is sorted.
 *   Groups: group g merges runs [group_off[g], group_off[g+1]) (device,
 *     groups+1 entries, group_off[0] = 0, group_off[groups] = k,
 *     1 <= groups <= k).
 * Output, n_out = sum of run sizes entries: group g's merged sequence occupies
 * the positions after all runs of earlier groups, in merged order:
 *   out_src[i] = (run << 32) | position within the run (may be NULL),
 *   out_id[i]  = fc_id of that element,
 *   out_lcp[i] = LCP with the previous string of the same group (0 for the
 *                group's first),
 *   out_len[i] = fc_len of that element (may be NULL).
 * Equal strings keep (run, position) order.  The runs are read in place; no
 * decoded copy is made.  out_cap is the capacity of each output array
 * (CAPACITY if n_out exceeds it); *n_out_host (host, may be NULL) receives
 * n_out.  The call reads the run bounds back (it synchronises the stream). */
int ss_lcp_merge(uint32_t k, const uint64_t *run_begin, const uint64_t *run_end, uint32_t groups,
                 const uint32_t *group_off, uint64_t n_fc, const uint32_t *fc_lcp,
                 const uint32_t *fc_len, const uint32_t *fc_id, const uint64_t *suf_off,
                 const uint8_t *suf, uint64_t *out_src, uint32_t *out_id, uint32_t *out_lcp,
                 uint32_t *out_len, uint64_t out_cap, uint64_t *n_out_host, void *ws, size_t ws_bytes,
                 void *stream);

/* ------------------------------------------------------------- suffixes */

/* Workspace bytes for ss_suffix_sort of a text of N bytes (about
 * 26 B + the ss_sort workspace per suffix). */
size_t ss_suffix_sort_workspace(uint64_t N);

/* Suffix sorting by sorting strings of equal length (the application
 * Section 6 names), space-efficiently: the N suffixes T[i, N) of one text
 * are never stored.  Prefix doubling over ranks: each step sorts one
 * equal-length string per suffix -- its pair (rank of its h-prefix, rank of
 * the h-prefix h bytes later) as 7 big-endian bytes (8 when N >= 2^28) --
 * with ss_sort and re-ranks, doubling h from 6 until every rank is distinct
 * (about log2(max LCP / 6) + 1 steps; one read-back per step).
 *   sa (out, N)  start of the k-th smallest suffix (a proper prefix sorts
 *                first; suffixes are distinct).
 *   lcp (out, N, nullable)  lcp[0] = 0, lcp[k] = LCP of the suffixes at k-1
 *                and k, by comparison (cost: the sum of the LCPs).
 *   steps_host (host, out, nullable)  sorting steps run.
 * TOO_LARGE if N >= 2^32 - 1. */
int ss_suffix_sort(const uint8_t *text, uint64_t N, uint32_t *sa, uint32_t *lcp, uint32_t *steps_host,
                   void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- graphs */

/* A launch sequence of library calls captured once from a stream and replayed
 * with one launch (a HIP graph).  Between ss_graph_begin(stream) and
 * ss_graph_end(stream, &g) the calling thread enqueues capturable calls on
 * `stream` (not the null stream); they are recorded, not run.  Capturable:
 * ss_sort_batch_device, ss_dist_exact, ss_dist_exact_bounded, ss_lcp,
 * ss_select_splitters, ss_bucket_bounds, ss_fc_decode_noalloc (no read-back,
 * no allocation).  Pointers and sizes are fixed at capture: a replay reads
 * whatever the captured buffers hold then.  Kernel profiling must be off.
 * ss_graph_launch enqueues one replay on `stream`; replays of one graph must
 * not overlap (they share the captured buffers). */
typedef struct ss_graph_s *ss_graph;
int ss_graph_begin(void *stream);
int ss_graph_end(void *stream, ss_graph *out);
int ss_graph_launch(ss_graph g, void *stream);
size_t ss_graph_nodes(ss_graph g); /* kernel and other nodes of the graph */
void ss_graph_destroy(ss_graph g);

/* ------------------------------------------------------------ profiling */

/* Opt-in kernel timing for measurement (not part of the method).  While
 * enabled, the library records a HIP event pair on the launch stream around
 * every launch of its main kernels, together with the launch's algorithmic
 * byte count (the bytes the step must move: inputs read once, outputs written
 * once; each kernel's figure is stated where it is launched).  Enabling clears
 * earlier records.  Records are process-wide; use from one thread. */
void ss_profile_enable(int on);

/* Record only the launches of kernel `name` (NULL or "": all).  Fewer event
 * pairs in a timed region cost less host time.  Set it while no library call
 * is running. */
void ss_profile_only(const char *name);

/* Totals for kernel `name` over the records so far: summed event time (ms),
 * summed algorithmic bytes and number of launches (synchronises the recorded
 * events).  Returns SS_OK, or SS_ERR_INVALID_ARG if nothing was recorded. */
int ss_profile_query(const char *name, double *ms, double *bytes, uint32_t *launches);

/* Comma-separated names of the kernels recorded so far, into a host buffer of
 * `cap` bytes.  Returns the length needed (excluding the terminator). */
size_t ss_profile_names(char *buf, size_t cap);

/* ------------------------------------------------------------- tuning */

/* Tunable launch parameters (chosen by the autotuner; defaults are safe).
 *   SS_TUNE_SMALL_MAX  segments up to this many strings are sorted in LDS
 *                      (128, 256, 512 or 1024; default 1024).
 *   SS_TUNE_TILE       elements per workgroup in radix passes (1024..16384,
 *                      power of two; default 4096).
 *   SS_TUNE_DIGIT_BITS radix digit width: 8 (a level per key byte, 256
 *                      buckets) or 11 (six levels per 64-bit key, 2048
 *                      buckets); 11 takes effect only with a tile >= 4096 and
 *                      SMALL_MAX >= 512, else 8 is used (default 8).
 *   SS_TUNE_DEDUP      prefix doubling's duplicate detection: 0 = a global
 *                      hash table (default); 1 = buckets of keys counted in
 *                      LDS for lists of 2^16..2^26 keys, the table otherwise;
 *                      2 = buckets for every list up to 2^26 keys.
 *   SS_TUNE_DEDUP_LOG_BUCKETS  log2 of the number of buckets (1..14; 0 = by
 *                      the list length, about 2048 keys a bucket; default 0).
 * Results never depend on the tuning.  Returns the previous value, or
 * SS_ERR_INVALID_ARG. */
#define SS_TUNE_SMALL_MAX 1
#define SS_TUNE_TILE 2
#define SS_TUNE_DIGIT_BITS 3
#define SS_TUNE_DEDUP 4
#define SS_TUNE_DEDUP_LOG_BUCKETS 5
int ss_set_tuning(int param, int value);

#ifdef __cplusplus
}
#endif
#endif /* STRSORT_H */
