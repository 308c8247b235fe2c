/*
 * CPU oracle for the string-sorting hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct single-threaded C.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg load this library; the GPU
 * product path never links, calls or includes anything from here, and this
 * file shares no code, header, table or constant generator with it.
 *
 * Notation follows "Scalable Distributed String Sorting" (Kurpicz, Mehnert,
 * Sanders, Schimek):
 *   - a string array S = [s_0..s_{n-1}] given as a character array plus
 *     offsets (Section 2, "String Properties and Input Format");
 *   - lcp(s, t) and the LCP array [h_0, h_1, ..] with h_i = lcp(s_{i-1}, s_i)
 *     over the sorted order (Section 2);
 *   - the distinguishing prefix dist(s) and D = sum dist (Section 2);
 *   - dist_approx(s) >= dist(s) by prefix doubling over prefix hashes with
 *     duplicate detection (Section 4, and the proof outline in Appendix C);
 *   - buckets B^j = { s : f_j < s <= f_{j+1} } (Section 3, step 1);
 *   - LCP compression: a common prefix with the predecessor is sent only once
 *     (Section 2, "Algorithmic Building Blocks");
 *   - LCP-aware merging of sorted runs (Section 2 / Section 3, step 3): the
 *     oracle computes the merge result by its plain definition (a stable sort of
 *     the union), which the LCP loser tree reaches faster.
 *
 * Readings where the paper is silent:
 *   R1 strings carry explicit lengths; a string that is a proper prefix of
 *      another is smaller (the end sentinel sorts below every byte, Section 2),
 *      and lengths / dist count bytes only (no sentinel).
 *   R2 lcp counts equal leading bytes, at most the shorter length.
 *   R3 equal strings are allowed; ties are broken by input index (stable).
 *   R4 h_0 = 0.
 *   R5 dist(s) = min(len(s), 1 + max over t != s of lcp(s, t)); the maximum
 *      is attained at a sorted neighbour, so with lcp[n] := 0
 *      dist(s_perm[i]) = min(len, 1 + max(lcp[i], lcp[i+1])).
 *   R6 initial doubling length l_0 (paper: Theta(log p / log sigma)) is a
 *      parameter, a positive multiple of 4; the workloads use 8.
 *   R7 the hash (paper: "a hash" / "random hash function") is frozen as
 *      Karp-Rabin modulo the Mersenne prime 2^61-1 over 4-byte little-endian
 *      limbs with the prefix length appended as a final digit (see kr_key).
 *   R9 uniqueness is decided among the strings still active in the round;
 *      strings with len <= l still take part as keys in that round.
 *   R10 ties with a splitter go to the lower bucket (the "<=" of Section 3).
 *   R11 front-coding format: per bucket, e_i = 0 at the bucket start, else the
 *      LCP with the predecessor; d_i = len (full strings) or dist_approx
 *      (distinguishing prefixes only, Section 4); literal bytes s[e_i, d_i).
 *   R12 merge ties are broken by (run, position).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- strings */

static int str_cmp(const uint8_t *a, uint64_t la, const uint8_t *b, uint64_t lb)
{
    /* R1: unsigned byte order, a proper prefix sorts first. */
    uint64_t m = la < lb ? la : lb;
    for (uint64_t i = 0; i < m; i++) {
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    }
    if (la == lb) return 0;
    return la < lb ? -1 : 1;
}

static uint64_t str_lcp(const uint8_t *a, uint64_t la, const uint8_t *b, uint64_t lb)
{
    /* R2: number of equal leading bytes. */
    uint64_t m = la < lb ? la : lb, i = 0;
    while (i < m && a[i] == b[i]) i++;
    return i;
}

#define SP(i) (bytes + off[(i)])
#define SL(i) (off[(i) + 1] - off[(i)])
#define SLEN(i) (off[(i) + 1] - off[(i)])

/* Order of (string, input index): the stable sorted order of R3. */
static int idx_less(const uint8_t *bytes, const uint64_t *off, uint32_t x, uint32_t y)
{
    int c = str_cmp(SP(x), SL(x), SP(y), SL(y));
    if (c) return c < 0;
    return x < y;
}

static void msort_idx(const uint8_t *bytes, const uint64_t *off, uint32_t *a, uint32_t *tmp,
                      uint64_t n)
{
    if (n < 2) return;
    uint64_t h = n / 2;
    msort_idx(bytes, off, a, tmp, h);
    msort_idx(bytes, off, a + h, tmp, n - h);
    uint64_t i = 0, j = h, k = 0;
    while (i < h && j < n) {
        if (idx_less(bytes, off, a[j], a[i])) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, n * sizeof(uint32_t));
}

/* Sorting (Section 3, "Initialization"): perm[i] = input index of the i-th
 * smallest string, ties by input index.  Returns 0, or -1 on allocation failure. */
int or_sort(const uint8_t *bytes, const uint64_t *off, uint64_t n, uint32_t *perm)
{
    for (uint64_t i = 0; i < n; i++) perm[i] = (uint32_t)i;
    if (n < 2) return 0;
    uint32_t *tmp = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!tmp) return -1;
    msort_idx(bytes, off, perm, tmp, n);
    free(tmp);
    return 0;
}

/* LCP array (Section 2): lcp[0] = 0 (R4), lcp[i] = lcp(s_perm[i-1], s_perm[i]). */
void or_lcp(const uint8_t *bytes, const uint64_t *off, uint64_t n, const uint32_t *perm,
            uint32_t *lcp)
{
    if (n == 0) return;
    lcp[0] = 0;
    for (uint64_t i = 1; i < n; i++) {
        uint32_t a = perm[i - 1], b = perm[i];
        lcp[i] = (uint32_t)str_lcp(SP(a), SL(a), SP(b), SL(b));
    }
}

/* Exact distinguishing prefix (Section 2, reading R5), indexed by input index. */
void or_dist_exact(const uint64_t *off, uint64_t n, const uint32_t *perm, const uint32_t *lcp,
                   uint32_t *dist)
{
    for (uint64_t i = 0; i < n; i++) {
        uint64_t a = lcp[i];
        uint64_t b = (i + 1 < n) ? lcp[i + 1] : 0;
        uint64_t m = (a > b ? a : b) + 1;
        uint64_t len = SL(perm[i]);
        dist[perm[i]] = (uint32_t)(m < len ? m : len);
    }
}

/* Brute force of R5's first form (every pair); for tiny inputs only. */
void or_dist_bruteforce(const uint8_t *bytes, const uint64_t *off, uint64_t n, uint32_t *dist)
{
    for (uint64_t i = 0; i < n; i++) {
        uint64_t best = 0;
        for (uint64_t j = 0; j < n; j++) {
            if (j == i) continue;
            uint64_t l = str_lcp(SP(i), SL(i), SP(j), SL(j));
            if (l > best) best = l;
        }
        uint64_t m = (n > 1) ? best + 1 : 1;
        dist[i] = (uint32_t)(m < SL(i) ? m : SL(i));
    }
}

/* ------------------------------------------------------------------ hash */

#define KR_P ((uint64_t)0x1FFFFFFFFFFFFFFFull) /* 2^61 - 1 */
#define KR_B ((uint64_t)0x0B3C4D5E6F708192ull) /* fixed base, 2^32 <= B < p */

static uint64_t mulmod_p(uint64_t a, uint64_t b)
{
    unsigned __int128 x = (unsigned __int128)a * b;
    return (uint64_t)(x % KR_P);
}

/* R7: Karp-Rabin key of the m-byte prefix s[0, m).  The prefix is cut into
 * 4-byte little-endian limbs (the last one zero-padded), C = sum_j limb_j *
 * B^(q-1-j) mod p by Horner's rule, and the key is (C * B + m) mod p. */
uint64_t or_kr_key(const uint8_t *s, uint64_t m)
{
    uint64_t C = 0;
    for (uint64_t j = 0; j < m; j += 4) {
        uint64_t limb = 0;
        for (uint64_t t = 0; t < 4; t++) {
            uint64_t byte = (j + t < m) ? s[j + t] : 0;
            limb |= byte << (8 * t);
        }
        C = (mulmod_p(C, KR_B) + limb) % KR_P;
    }
    return (mulmod_p(C, KR_B) + m) % KR_P;
}

static uint64_t mask_key(uint64_t key, uint32_t hash_bits)
{
    if (hash_bits >= 64) return key;
    return key & ((1ull << hash_bits) - 1);
}

typedef struct { uint64_t key; uint32_t idx; uint32_t m; } kr_item;

static int item_cmp(const void *x, const void *y)
{
    const kr_item *a = (const kr_item *)x, *b = (const kr_item *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Approximate distinguishing prefixes by prefix doubling (Section 4 and the
 * proof outline of Appendix C), one device's share with exact duplicate
 * detection on the hash values (Appendix B: sort (hash, index) pairs, then a
 * scan finds the duplicates).
 *
 * Round t tests prefix length l_t = init_len * 2^t.  Every active string s
 * gets key H(s[0, min(l_t, len))); it is finished when its key is unique among
 * the active strings or when len <= l_t, with dist_approx = min(l_t, len).
 * Outputs are indexed by input index.  *rounds receives the number of rounds,
 * *collisions the number of adjacent equal-key pairs whose prefixes differ.
 * Returns 0, -1 on allocation failure, -2 on a bad init_len. */
int or_dist_prefix(const uint8_t *bytes, const uint64_t *off, uint64_t n, uint32_t init_len,
                   uint32_t hash_bits, uint32_t *dist, uint32_t *rounds, uint64_t *collisions)
{
    if (init_len == 0 || (init_len % 4) != 0) return -2;
    uint32_t *act = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    kr_item *it = (kr_item *)malloc((n ? n : 1) * sizeof(kr_item));
    if (!act || !it) { free(act); free(it); return -1; }
    uint64_t na = n, coll = 0;
    for (uint64_t i = 0; i < n; i++) act[i] = (uint32_t)i;
    uint64_t l = init_len;
    uint32_t t = 0;
    while (na > 0) {
        t++;
        for (uint64_t a = 0; a < na; a++) {
            uint32_t s = act[a];
            uint64_t len = SL(s), m = len < l ? len : l;
            it[a].key = mask_key(or_kr_key(SP(s), m), hash_bits);
            it[a].idx = s;
            it[a].m = (uint32_t)m;
        }
        qsort(it, na, sizeof(kr_item), item_cmp);
        uint64_t keep = 0;
        for (uint64_t a = 0; a < na; a++) {
            int dup = (a > 0 && it[a - 1].key == it[a].key) ||
                      (a + 1 < na && it[a + 1].key == it[a].key);
            if (a > 0 && it[a - 1].key == it[a].key) {
                const kr_item *p = &it[a - 1], *q = &it[a];
                if (p->m != q->m || memcmp(SP(p->idx), SP(q->idx), q->m) != 0) coll++;
            }
            uint32_t s = it[a].idx;
            uint64_t len = SL(s);
            if (!dup || len <= l) dist[s] = (uint32_t)(len < l ? len : l);
            else act[keep++] = s;
        }
        na = keep;
        l *= 2;
    }
    free(act);
    free(it);
    if (rounds) *rounds = t;
    if (collisions) *collisions = coll;
    return 0;
}

/* ------------------------------------------------------- splitters, buckets */

/* One-device reading of regular sampling (Section 3.1, f_j = V[j|V|/r - 1])
 * with V = the whole sorted local array: f_j = s_perm[ceil(j n / r) - 1] for
 * j = 1..r-1.  ids[j-1] receives the input index of f_j.  Returns 0 or -1. */
int or_select_splitters(uint64_t n, const uint32_t *perm, uint32_t r, uint32_t *ids)
{
    if (n == 0 || r == 0) return -1;
    for (uint64_t j = 1; j < r; j++) {
        uint64_t c = (j * n + r - 1) / r;
        ids[j - 1] = perm[c - 1];
    }
    return 0;
}

/* Character-based regular sampling (Section 3.1, "Character-Based Sampling";
 * Appendix A): samples are drawn at equally spaced positions of the sorted
 * array's character array and each sampled position is shifted back to the
 * beginning of the string that contains it.  One array's form with r - 1
 * samples: with C_k = characters of the strings at sorted positions < k and
 * N = C_n, sample j (j = 1..r-1) is at character position
 * x_j = ceil(j N / r) - 1 (the character analogue of f_j = V[j|V|/r - 1]),
 * and ids[j-1] = perm[k] for the string k with C_k <= x_j < C_{k+1}.
 * Characters are the full lengths, or the given per-string counts `w`
 * (indexed by input index; e.g. approximate distinguishing prefixes, the
 * characters prefix doubling keeps).  N = 0 (no characters) samples the
 * first string.  Returns 0, or -1 if n == 0 or r == 0. */
int or_select_splitters_chars(uint64_t n, const uint32_t *perm, const uint64_t *off, const uint32_t *w,
                              uint32_t r, uint32_t *ids)
{
    if (n == 0 || r == 0) return -1;
    uint64_t N = 0;
    for (uint64_t k = 0; k < n; k++) N += w ? w[perm[k]] : SLEN(perm[k]);
    for (uint32_t j = 1; j < r; j++) {
        if (N == 0) {
            ids[j - 1] = perm[0];
            continue;
        }
        uint64_t x = ((uint64_t)j * N + r - 1) / r - 1;
        uint64_t C = 0, k = 0;
        for (;; k++) {
            uint64_t c = w ? w[perm[k]] : SLEN(perm[k]);
            if (x < C + c) break;  /* (x < N, so some string contains it) */
            C += c;
        }
        ids[j - 1] = perm[k];
    }
    return 0;
}

/* Buckets (Section 3, step 1): bounds[0] = 0, bounds[r] = n and
 * bounds[j] = #{ i : s_perm[i] <= f_j } for the r-1 splitters f_1..f_{r-1}
 * given as a string array (sb, soff).  Plain count (R10). */
void or_bucket_bounds(const uint8_t *bytes, const uint64_t *off, uint64_t n,
                      const uint32_t *perm, const uint8_t *sb, const uint64_t *soff, uint32_t r,
                      uint64_t *bounds)
{
    bounds[0] = 0;
    for (uint32_t j = 1; j < r; j++) {
        const uint8_t *f = sb + soff[j - 1];
        uint64_t lf = soff[j] - soff[j - 1], c = 0;
        for (uint64_t i = 0; i < n; i++) {
            uint32_t s = perm[i];
            if (str_cmp(SP(s), SL(s), f, lf) <= 0) c++;
        }
        bounds[j] = c;
    }
    bounds[r] = n;
}

/* ----------------------------------------------------------- front coding */

/* LCP compression (Section 2) in format R11.  For each bucket j and sorted
 * position i in [bounds[j], bounds[j+1]): e_i = 0 at the bucket start else
 * lcp[i]; d_i = dist[perm[i]] if dist is given (distinguishing prefixes only,
 * Section 4) else len; id_i = perm[i]; literal bytes s[e_i, d_i) are appended
 * in order and suf_off[i] is their start (suf_off[n] = total).
 * Returns the total number of literal bytes, or -1 if some e_i > d_i. */
int64_t or_fc_encode(const uint8_t *bytes, const uint64_t *off, uint64_t n, const uint32_t *perm,
                     const uint32_t *lcp, const uint32_t *dist, const uint64_t *bounds, uint32_t r,
                     uint32_t *fc_lcp, uint32_t *fc_len, uint32_t *fc_id, uint64_t *suf_off,
                     uint8_t *suf)
{
    uint64_t pos = 0;
    for (uint32_t j = 0; j < r; j++) {
        for (uint64_t i = bounds[j]; i < bounds[j + 1]; i++) {
            uint32_t s = perm[i];
            uint64_t e = (i == bounds[j]) ? 0 : lcp[i];
            uint64_t d = dist ? dist[s] : SL(s);
            if (e > d) return -1;
            fc_lcp[i] = (uint32_t)e;
            fc_len[i] = (uint32_t)d;
            fc_id[i] = s;
            suf_off[i] = pos;
            memcpy(suf + pos, SP(s) + e, d - e);
            pos += d - e;
        }
    }
    suf_off[n] = pos;
    return (int64_t)pos;
}

/* Decoding: within a run, string i = the first e_i bytes of string i-1,
 * followed by its literal bytes.  out_off[n+1] are the decoded offsets. */
void or_fc_decode(uint32_t k, const uint64_t *run_off, const uint32_t *fc_lcp,
                  const uint32_t *fc_len, const uint64_t *suf_off, const uint8_t *suf, uint64_t n,
                  uint64_t *out_off, uint8_t *out)
{
    out_off[0] = 0;
    for (uint64_t i = 0; i < n; i++) out_off[i + 1] = out_off[i] + fc_len[i];
    for (uint32_t j = 0; j < k; j++) {
        for (uint64_t i = run_off[j]; i < run_off[j + 1]; i++) {
            uint64_t e = fc_lcp[i], d = fc_len[i];
            if (i > run_off[j]) memcpy(out + out_off[i], out + out_off[i - 1], e);
            memcpy(out + out_off[i] + e, suf + suf_off[i], d - e);
        }
    }
}

/* ----------------------------------------------------------------- merging */

typedef struct {
    const uint8_t *b;
    const uint64_t *o;
    const uint64_t *run_off;
} merge_ctx;

static int merge_less(const merge_ctx *c, uint64_t x, uint64_t y)
{
    /* x, y index the concatenated runs; order (string, run, position) (R12).
     * Concatenation index order equals (run, position) order. */
    int r = str_cmp(c->b + c->o[x], c->o[x + 1] - c->o[x], c->b + c->o[y], c->o[y + 1] - c->o[y]);
    if (r) return r < 0;
    return x < y;
}

static void msort_merge(const merge_ctx *c, uint64_t *a, uint64_t *tmp, uint64_t n)
{
    if (n < 2) return;
    uint64_t h = n / 2;
    msort_merge(c, a, tmp, h);
    msort_merge(c, a + h, tmp, n - h);
    uint64_t i = 0, j = h, k = 0;
    while (i < h && j < n) {
        if (merge_less(c, a[j], a[i])) tmp[k++] = a[j++];
        else tmp[k++] = a[i++];
    }
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, n * sizeof(uint64_t));
}

/* Merging k sorted front-coded runs (Section 3, step 3) by the plain
 * definition: decode, stable-sort the union by (string, run, position),
 * recompute the LCP of merged neighbours.  out_src[i] = (run << 32) | pos,
 * out_id[i] = fc_id of that element, out_lcp[i] = its LCP with the previous
 * output (0 for i = 0).  Returns 0 or -1 on allocation failure. */
int or_merge(uint32_t k, const uint64_t *run_off, const uint32_t *fc_lcp, const uint32_t *fc_len,
             const uint32_t *fc_id, const uint64_t *suf_off, const uint8_t *suf, uint64_t n,
             uint64_t *out_src, uint32_t *out_id, uint32_t *out_lcp)
{
    uint64_t total = 0;
    for (uint64_t i = 0; i < n; i++) total += fc_len[i];
    uint64_t *doff = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    uint8_t *dec = (uint8_t *)malloc(total ? total : 1);
    uint64_t *ord = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t *tmp = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    if (!doff || !dec || !ord || !tmp) {
        free(doff); free(dec); free(ord); free(tmp);
        return -1;
    }
    or_fc_decode(k, run_off, fc_lcp, fc_len, suf_off, suf, n, doff, dec);
    for (uint64_t i = 0; i < n; i++) ord[i] = i;
    merge_ctx c = {dec, doff, run_off};
    msort_merge(&c, ord, tmp, n);
    for (uint64_t i = 0; i < n; i++) {
        uint64_t g = ord[i];
        uint32_t run = 0;
        while (!(g >= run_off[run] && g < run_off[run + 1])) run++;
        out_src[i] = ((uint64_t)run << 32) | (g - run_off[run]);
        out_id[i] = fc_id[g];
        if (i == 0) out_lcp[i] = 0;
        else {
            uint64_t p = ord[i - 1];
            out_lcp[i] = (uint32_t)str_lcp(dec + doff[p], doff[p + 1] - doff[p], dec + doff[g],
                                           doff[g + 1] - doff[g]);
        }
    }
    free(doff); free(dec); free(ord); free(tmp);
    return 0;
}

/* ------------------------------------------------------------ suffixes */

/* Suffix sorting, the application of string sorting the paper names as
 * future work (Section 6): the suffixes T[i, N) of one text, which overlap
 * and are never stored as separate strings, in lexicographic order (a suffix
 * that is a prefix of another sorts first; suffixes are distinct, so there
 * are no ties).  Plain definition: sort the start positions with a
 * suffix comparator.  sa (out, N) = start of the k-th smallest suffix;
 * lcp (out, N, nullable) = lcp[0] = 0, lcp[k] = lcp(T[sa[k-1], N), T[sa[k], N)).
 * Returns 0, or -1 on allocation failure. */
static const uint8_t *g_sfx_text;
static uint64_t g_sfx_n;

static int sfx_cmp(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return str_cmp(g_sfx_text + a, g_sfx_n - a, g_sfx_text + b, g_sfx_n - b);
}

int or_suffix_sort(const uint8_t *text, uint64_t N, uint32_t *sa, uint32_t *lcp)
{
    for (uint64_t i = 0; i < N; i++) sa[i] = (uint32_t)i;
    g_sfx_text = text;  /* (single-threaded oracle) */
    g_sfx_n = N;
    qsort(sa, N, sizeof(uint32_t), sfx_cmp);
    if (lcp && N > 0) {
        lcp[0] = 0;
        for (uint64_t k = 1; k < N; k++)
            lcp[k] = (uint32_t)str_lcp(text + sa[k - 1], N - sa[k - 1], text + sa[k], N - sa[k]);
    }
    return 0;
}

/* Check of a claimed suffix array at any size: sa must be a permutation of
 * 0..N-1 with every adjacent pair of suffixes in order, and lcp (nullable)
 * exact for every pair.  Time O(N + sum of the LCPs).  Returns -1 when all
 * holds, -2 if sa is not a permutation, else the first bad position. */
int64_t or_check_suffixes(const uint8_t *text, uint64_t N, const uint32_t *sa, const uint32_t *lcp)
{
    uint8_t *seen = (uint8_t *)calloc(N ? N : 1, 1);
    if (!seen) return -3;
    for (uint64_t k = 0; k < N; k++) {
        if (sa[k] >= N || seen[sa[k]]) { free(seen); return -2; }
        seen[sa[k]] = 1;
    }
    free(seen);
    if (lcp && N > 0 && lcp[0] != 0) return 0;
    for (uint64_t k = 1; k < N; k++) {
        const uint64_t a = sa[k - 1], b = sa[k];
        if (str_cmp(text + a, N - a, text + b, N - b) >= 0) return (int64_t)k;
        if (lcp && lcp[k] != (uint32_t)str_lcp(text + a, N - a, text + b, N - b)) return (int64_t)k;
    }
    return -1;
}

/* ---------------------------------------------------------------- checking */

/* Full check of a claimed sort + LCP result at any size, in linear time:
 * perm must be a permutation of 0..n-1, every adjacent pair must be in
 * (string, index) order (so the order is the unique stable sorted order) and
 * lcp must equal the brute-force LCP of every adjacent pair (lcp may be NULL).
 * Returns -1 when all holds, -2 if perm is not a permutation, otherwise the
 * first sorted position whose order or LCP is wrong. */
int64_t or_check_sorted(const uint8_t *bytes, const uint64_t *off, uint64_t n,
                        const uint32_t *perm, const uint32_t *lcp)
{
    uint8_t *seen = (uint8_t *)calloc(n ? n : 1, 1);
    if (!seen) return -3;
    for (uint64_t i = 0; i < n; i++) {
        if (perm[i] >= n || seen[perm[i]]) { free(seen); return -2; }
        seen[perm[i]] = 1;
    }
    free(seen);
    if (lcp && n > 0 && lcp[0] != 0) return 0;
    for (uint64_t i = 1; i < n; i++) {
        uint32_t a = perm[i - 1], b = perm[i];
        if (!idx_less(bytes, off, a, b)) return (int64_t)i;
        if (lcp && lcp[i] != (uint32_t)str_lcp(SP(a), SL(a), SP(b), SL(b))) return (int64_t)i;
    }
    return -1;
}
