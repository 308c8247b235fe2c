// Front-coding decode and LCP-aware k-way merge of sorted runs (Section 3,
// step 3; the LCP-aware merge building block of Section 2).
//
// Decode.  Within a run, string i equals the first e_i bytes of string i-1
// followed by its literal.  Its bytes [e_i, d_i) are its own literal; bytes
// [e_j, e_i) with j = psv(i) = the nearest earlier position with e_j < e_i are
// string j's literal, and so on down the psv chain to an e = 0 position (every
// run starts with e = 0).  psv is found by a min-tree search: inside each
// 1024-element block on a tree in LDS, else on a binary tree of the block
// minima (climb to the nearest left subtree holding a smaller value, descend to
// its rightmost such block, then its rightmost such 16-element chunk).  Each output 16-byte word then walks
// the chain of its string.
//
// Merge.  The paper merges r runs with an LCP loser tree.  Here the runs are
// merged pairwise in log2 k levels; each level is split into fixed-size output
// ranges by merge-path co-ranking, and every thread merges its range with the
// LCP rule: with h_a = lcp(last, a) and h_b = lcp(last, b), the larger of h_a,
// h_b decides without touching characters, and only on equality are the
// strings compared from h on.
#include <string.h>

#include <algorithm>
#include <vector>

#include <mutex>

#include "common.hpp"

#define PSV_NONE 0xFFFFFFFFu

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

// p[0..count) = v (a kernel rather than hipMemsetAsync, so that a captured
// graph holds no memset node).
__global__ void k_fill_u32(u32 *p, u32 v, u32 count)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

#define PB 1024  // psv block (one workgroup)
#define PC 16    // chunk whose minimum is kept for the far search
#define PCB (PB / PC)

// psv inside each block of PB entries (PSV_NONE if the answer lies before the
// block).  The block minimum goes to leaf P + block of the tree T, the minima
// of its PC-entry chunks to cm[block * PCB ..].  This and the kernels below do
// nothing when `need` is given and points to zero.
__global__ __launch_bounds__(PB) void k_psv_block(const u32 *e, u32 n, u32 *psv, u32 *T, u32 P, u32 *cm,
                                                 u32 *farl, u32 *fcnt, const u32 *need)
{
    if (need && *need == 0) return;
    __shared__ u32 t[2 * PB];  // heap: node x has children 2x, 2x+1; leaves PB..2PB-1
    const u32 b0 = blockIdx.x * PB;
    const u32 i = b0 + threadIdx.x;
    const u32 v = i < n ? e[i] : 0xFFFFFFFFu;
    t[PB + threadIdx.x] = v;
    __syncthreads();
    for (u32 c = PB / 2; c >= 1; c >>= 1) {
        if (threadIdx.x < c) {
            const u32 x = c + threadIdx.x;
            const u32 a = t[2 * x], b = t[2 * x + 1];
            t[x] = a < b ? a : b;
        }
        __syncthreads();
    }
    bool far = false;  // the answer lies before this block: left to k_psv_far
    if (i < n) {
        u32 res = PSV_NONE;
        if (v > 0) {
            u32 x = PB + threadIdx.x;
            bool found = false;
            while (x > 1) {
                if ((x & 1) && t[x - 1] < v) {
                    x = x - 1;
                    found = true;
                    break;
                }
                x >>= 1;
            }
            if (found) {
                while (x < PB) {
                    x = 2 * x + 1;
                    if (t[x] >= v) x--;
                }
                res = b0 + (x - PB);
            }
            far = !found;
        }
        psv[i] = res;
    }
    // this block's far entries, compacted to farl[b0 ..], their count in fcnt[block]
    __shared__ u32 wcnt[PB / 64];
    const u64 fm = __ballot(far);
    const u32 wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wcnt[wid] = (u32)__popcll(fm);
    __syncthreads();
    u32 wb = 0;
    for (u32 q = 0; q < wid; q++) wb += wcnt[q];
    if (far) farl[b0 + wb + (u32)__popcll(fm & lanemask_lt())] = i;
    if (threadIdx.x == 0) {
        u32 tot = 0;
        for (u32 q = 0; q < PB / 64; q++) tot += wcnt[q];
        fcnt[blockIdx.x] = tot;
    }
    if (threadIdx.x == 0) T[P + blockIdx.x] = t[1];
    if (threadIdx.x < PCB) cm[(u64)blockIdx.x * PCB + threadIdx.x] = t[PCB + threadIdx.x];
}

// Internal nodes of the tree T: each workgroup takes up to 512 nodes of one
// level (m nodes, indices m..2m-1) and writes `lv` levels above them.
__global__ __launch_bounds__(256) void k_tree_up(u32 *T, u32 m, u32 lv, const u32 *need)
{
    if (need && *need == 0) return;
    __shared__ u32 s[512];
    const u32 cnt = m < 512 ? m : 512;
    const u32 base = m + blockIdx.x * cnt;
    for (u32 q = threadIdx.x; q < cnt; q += 256) s[q] = T[base + q];
    __syncthreads();
    u32 c = cnt, b = base;
    for (u32 L = 0; L < lv; L++) {
        c >>= 1;
        b >>= 1;
        u32 v = 0;
        if (threadIdx.x < c) {
            const u32 x = s[2 * threadIdx.x], y = s[2 * threadIdx.x + 1];
            v = x < y ? x : y;
        }
        __syncthreads();
        if (threadIdx.x < c) {
            s[threadIdx.x] = v;
            T[b + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

// psv for positions whose answer lies before their block: nearest left
// subtree of T with a smaller minimum, its rightmost such block, that block's
// rightmost such chunk, that chunk's rightmost such entry.
__device__ __forceinline__ void psv_far_one(const u32 *e, const u32 *T, u32 P, const u32 *cm, u32 i, u32 n,
                                            u32 *psv)
{
    const u32 v = e[i];
    u32 x = P + i / PB;
    bool found = false;
    while (x > 1) {
        if ((x & 1) && T[x - 1] < v) {
            x = x - 1;
            found = true;
            break;
        }
        x >>= 1;
    }
    if (!found) return;  // malformed input (no e = 0 before): stays PSV_NONE
    while (x < P) {
        x = 2 * x + 1;
        if (T[x] >= v) x--;
    }
    const u32 blk = x - P;
    const uint4 *c4 = (const uint4 *)(cm + (u64)blk * PCB);  // 256-byte aligned workspace
    uint4 w[PCB / 4];
#pragma unroll
    for (int q = 0; q < PCB / 4; q++) w[q] = c4[q];
    int c = -1;
#pragma unroll
    for (int q = 0; q < PCB / 4; q++) {
        if (w[q].x < v) c = 4 * q;
        if (w[q].y < v) c = 4 * q + 1;
        if (w[q].z < v) c = 4 * q + 2;
        if (w[q].w < v) c = 4 * q + 3;
    }
    // the block minimum is < v, so some chunk qualifies (c >= 0), and that
    // chunk's entries all lie below n (padding entries are all-ones)
    const u32 lo = blk * PB + (u32)c * PC;
    u32 ev[PC];
#pragma unroll
    for (int q = 0; q < PC; q++) ev[q] = (lo + q < n) ? e[lo + q] : 0xFFFFFFFFu;
    u32 r = lo;
#pragma unroll
    for (int q = 0; q < PC; q++)
        if (ev[q] < v) r = lo + (u32)q;
    psv[i] = r;
}

// Workgroup b takes the far entries k_psv_block b left, packed at
// farl[b*PB ..] (fcnt[b] of them); each walk is a chain of dependent loads,
// so packing keeps the walks of a block in as few wavefronts as possible.
__global__ __launch_bounds__(256) void k_psv_far(const u32 *e, const u32 *T, u32 P, const u32 *cm, const u32 *farl,
                                                 const u32 *fcnt, u32 n, u32 *psv, const u32 *need)
{
    if (need && *need == 0) return;
    const u32 cnt = fcnt[blockIdx.x];
    const u32 *lst = farl + (u64)blockIdx.x * PB;
    for (u32 q = threadIdx.x; q < cnt; q += blockDim.x) psv_far_one(e, T, P, cm, lst[q], n, psv);
}

// Tree size (leaves) for n entries.
static u32 psv_leaves(u64 n)
{
    const u64 nb = ceil_div(n, PB);
    u32 P = 1;
    while (P < nb) P <<= 1;
    return P;
}

// psv of every entry of e[0..n) (n >= 1).  T holds 2 * psv_leaves(n) words,
// cm psv_leaves(n) * PCB words (256-byte aligned).  Skipped on the device
// when `need` is given and points to zero.
static int psv_build(const u32 *e, u64 n, u32 *psv, u32 *T, u32 *cm, u32 *farl, u32 *fcnt, hipStream_t st,
                     const u32 *need = nullptr)
{
    if (n == 0) return SS_OK;
    const u32 nb = (u32)ceil_div(n, PB);
    const u32 P = psv_leaves(n);
    if (P > nb) {
        k_fill_u32<<<(unsigned)ceil_div(P - nb, 256), 256, 0, st>>>(T + P + nb, 0xFFFFFFFFu, P - nb);
        SS_CHECK_LAUNCH();
    }
    {
        SS_PROF("k_psv_block", st, (double)n * 8.0);  // e in, psv out
        k_psv_block<<<nb, PB, 0, st>>>(e, (u32)n, psv, T, P, cm, farl, fcnt, need);
    }
    SS_CHECK_LAUNCH();
    for (u32 m = P; m > 1;) {
        u32 lv = 0;
        while (lv < 9 && (m >> lv) > 1) lv++;
        const u32 blocks = m > 512 ? m / 512 : 1;
        k_tree_up<<<blocks, 256, 0, st>>>(T, m, lv, need);
        SS_CHECK_LAUNCH();
        m >>= lv;
    }
    {
        // (far entries only: their value, the tree path, one chunk)
        SS_PROF("k_psv_far", st, 0.0);
        k_psv_far<<<nb, 256, 0, st>>>(e, T, P, cm, farl, fcnt, (u32)n, psv, need);
    }
    SS_CHECK_LAUNCH();
    return SS_OK;
}

#define DC_NT 256
#define DC_PER 16

// Decoded bytes of output chunk c0 .. c0 + DC_NT*DC_PER, 16 per thread, in
// output order (called by the whole workgroup; range is LDS).
__device__ __forceinline__ void decode_chunk(u64 c0, const u32 *e, const u32 *d, const u64 *suf_off, const u8 *suf,
                                             const u32 *psv, u32 n, const u64 *out_off, u64 total, u8 *out,
                                             u32 *range)
{
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
    if (q0 >= c1) return;  // (after the only barrier)
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

__global__ __launch_bounds__(DC_NT) void k_decode(const u32 *e, const u32 *d, const u64 *suf_off,
                                                  const u8 *suf, const u32 *psv, u32 n, const u64 *out_off,
                                                  u64 total, u8 *out)
{
    __shared__ u32 range[2];
    decode_chunk((u64)blockIdx.x * DC_NT * DC_PER, e, d, suf_off, suf, psv, n, out_off, total, out, range);
}

// The same with the total read on the device (out_off[n]) and the chunks
// taken in a grid-stride loop; nothing is written unless *status is 0.
__global__ __launch_bounds__(DC_NT) void k_decode_dev(const u32 *e, const u32 *d, const u64 *suf_off,
                                                      const u8 *suf, const u32 *psv, u32 n, const u64 *out_off,
                                                      const u32 *status, u8 *out)
{
    __shared__ u32 range[2];
    if (*status != 0) return;
    const u64 total = out_off[n];
    for (u64 c0 = (u64)blockIdx.x * DC_NT * DC_PER; c0 < total; c0 += (u64)gridDim.x * DC_NT * DC_PER) {
        decode_chunk(c0, e, d, suf_off, suf, psv, n, out_off, total, out, range);
        __syncthreads();  // range is rewritten by the next chunk
    }
}

// status = 0 (runs well formed, decoded bytes fit), 1 (malformed runs) or 2
// (more decoded bytes than cap).
__global__ void k_decode_status(const u32 *bad, const u64 *out_off, u32 n, u64 cap, u32 *status)
{
    *status = *bad ? 1u : (out_off[n] > cap ? 2u : 0u);
}

__global__ void k_widen(const u32 *d, u32 n, u64 *out)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = d[i];
}

struct DecWs {
    u32 *psv, *tree, *cmin, *bad, *far, *fcnt;
    u64 *scratch;
};

static void dec_layout(u64 n, DecWs *w, WsArena *a, WsCounter *c)
{
    const u64 nt = 2 * (u64)psv_leaves(n);
    if (a) {
        w->psv = a->take<u32>(n + 1);
        w->tree = a->take<u32>(nt);
        w->cmin = a->take<u32>(nt / 2 * PCB);
        w->bad = a->take<u32>(4);
        w->far = a->take<u32>(n + 1);
        w->fcnt = a->take<u32>(ceil_div(n, PB) + 1);
        w->scratch = a->take<u64>(ss_scan_scratch_elems<u64>(n + 1));
    } else {
        c->take<u32>(n + 1);
        c->take<u32>(nt);
        c->take<u32>(nt / 2 * PCB);
        c->take<u32>(4);
        c->take<u32>(n + 1);
        c->take<u32>(ceil_div(n, PB) + 1);
        c->take<u64>(ss_scan_scratch_elems<u64>(n + 1));
    }
}

static int decode_impl(u32 k, const u64 *run_off, const u32 *e, const u32 *d, const u64 *suf_off, const u8 *suf,
                       u64 n, u64 *out_off, u8 *out, u64 out_cap, DecWs &w, hipStream_t st)
{
    k_fill_u32<<<1, 64, 0, st>>>(w.bad, 0u, 1);
    SS_CHECK_LAUNCH();
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
    SS_TRY(psv_build(e, n, w.psv, w.tree, w.cmin, w.far, w.fcnt, st));
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

// ------------------------------------------------ allocation-free decode
//
// ss_fc_decode_noalloc keeps its scratch in one static device array per GPU
// (the code object's copy on each device) instead of a caller workspace.  In
// host code the array's name is only a stand-in: its device address is
// looked up once per device with hipGetSymbolAddress (on the call's first
// use of that device, with the device current) and only that address is
// passed to kernels.  Calls on one device share the array: calls that
// overlap on one GPU (different streams, or threads) race.

#define FCD_NOALLOC_SCRATCH_BYTES (36u << 20)
static __device__ __align__(256) unsigned char scratch[FCD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int FCD_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[FCD_MAX_DEVICES] = {};

int scratch_address(void **out)
{
    int dev = 0;
    SS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= FCD_MAX_DEVICES) {
        ss_set_error("device index %d beyond %d", dev, FCD_MAX_DEVICES);
        return SS_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            ss_set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
            return SS_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SS_OK;
}
}  // namespace

extern "C" int ss_fc_decode_noalloc(uint32_t k, const uint64_t *run_off, const uint32_t *fc_lcp,
                                    const uint32_t *fc_len, const uint64_t *suf_off, const uint8_t *suf,
                                    uint64_t n, uint64_t *out_offsets, uint8_t *out_bytes, uint64_t out_cap,
                                    uint32_t *status, void *stream)
{
    ss_clear_error();
    if (n > SS_FC_DECODE_NOALLOC_MAX) {
        ss_set_error("fc_decode_noalloc: n = %llu exceeds the limit of %u entries", (unsigned long long)n,
                     (unsigned)SS_FC_DECODE_NOALLOC_MAX);
        return SS_ERR_TOO_LARGE;
    }
    if (k == 0 || !run_off || !out_offsets || !status || (n > 0 && (!fc_lcp || !fc_len || !suf_off))) {
        ss_set_error("fc_decode_noalloc: bad arguments");
        return SS_ERR_INVALID_ARG;
    }
    if (ss_fc_decode_workspace(n) > FCD_NOALLOC_SCRATCH_BYTES) {  // (cannot happen below the limit)
        ss_set_error("fc_decode_noalloc: scratch too small for n = %llu", (unsigned long long)n);
        return SS_ERR_TOO_LARGE;
    }
    void *base = nullptr;
    SS_TRY(scratch_address(&base));
    hipStream_t st = (hipStream_t)stream;
    WsArena a(base, FCD_NOALLOC_SCRATCH_BYTES);
    DecWs w;
    dec_layout(n, &w, &a, nullptr);
    const u32 *e = fc_lcp, *d = fc_len;
    // w.bad starts at zero on every call (the array keeps the last call's contents)
    k_fill_u32<<<1, 64, 0, st>>>(w.bad, 0u, 1);
    SS_CHECK_LAUNCH();
    const u64 grid = ceil_div((n > k ? n : k) + 1, 256);
    k_check_runs<<<(unsigned)grid, 256, 0, st>>>(run_off, k, e, d, (u32)n, w.bad);
    SS_CHECK_LAUNCH();
    if (n > 0) {
        k_widen<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(d, (u32)n, out_offsets);
        SS_CHECK_LAUNCH();
    }
    SS_TRY(ss_scan_exclusive<u64>(out_offsets, out_offsets, n, w.scratch, st));
    k_decode_status<<<1, 1, 0, st>>>(w.bad, out_offsets, (u32)n, out_cap, status);
    SS_CHECK_LAUNCH();
    if (n == 0 || out_cap == 0) return SS_OK;
    // the psv chains only read e (any values are safe); bytes are decoded
    // only when the status is 0
    SS_TRY(psv_build(e, n, w.psv, w.tree, w.cmin, w.far, w.fcnt, st));
    const u64 chunks = ceil_div(out_cap, (u64)DC_NT * DC_PER);
    k_decode_dev<<<(unsigned)(chunks < 4096 ? chunks : 4096), DC_NT, 0, st>>>(e, d, suf_off, suf, w.psv, (u32)n,
                                                                            out_offsets, status, out_bytes);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

// ----------------------------------------------------------------- merge

// Read access to front-coded strings without decoding them: bytes [k, k+take)
// of string g are gathered piece by piece along its psv chain.
struct FcView {
    const u32 *e, *d, *psv;
    const u64 *suf_off;
    const u8 *suf;
    u64 sufN;
};

// The literal piece of front-coded string g that holds byte k (< d_g): the
// offset in suf of byte k, and how many of the string's bytes from k on lie
// in that literal (the chain element whose e is the first <= k, walking the
// psv chain from g; its literal covers bytes [e_j, e of the element after it
// toward g), or [e_g, d_g) for g itself).
__device__ __forceinline__ void fc_piece(const FcView &V, u32 g, u64 k, u64 *pos, u64 *avail)
{
    u32 j = g;
    u64 h = V.d[g];
    u32 ej = V.e[j];
    while (ej > k) {
        h = ej;
        j = V.psv[j];
        ej = V.e[j];
    }
    *pos = V.suf_off[j] + (k - ej);
    *avail = h - k;
}

// Three-way comparison of front-coded strings x and y from byte `from`
// (they agree on [0, from)); *lcp receives their LCP.  Merges call it where
// cached keys tie, in lockstep wavefronts where one lane's comparison holds
// up the others, so its chain of dependent loads is kept short: both
// strings' lengths, LCPs and literal offsets are loaded together; a string
// whose own literal holds byte `from` (the usual case) is read from there
// without a chain walk, otherwise its piece is found along its psv chain;
// the two pieces are then compared 32 bytes a round, every word of a round
// loaded before any is compared, until one piece ends.
#define FC_ROUND 4  // 8-byte words per comparison round

__device__ __forceinline__ int fc_cmp(const FcView &V, u32 x, u32 y, u64 from, u64 *lcp)
{
    const u64 lx = V.d[x], ly = V.d[y];
    const u32 ex = V.e[x], ey = V.e[y];
    const u64 sx = V.suf_off[x], sy = V.suf_off[y];
    const u64 m = lx < ly ? lx : ly;
    u64 i = from < m ? from : m;
    u64 px = 0, ax = 0, py = 0, ay = 0;
    if (i < m) {
        if (ex <= i) { px = sx + (i - ex); ax = lx - i; }
        else fc_piece(V, x, i, &px, &ax);
        if (ey <= i) { py = sy + (i - ey); ay = ly - i; }
        else fc_piece(V, y, i, &py, &ay);
    }
    while (i < m) {
        if (ax == 0) fc_piece(V, x, i, &px, &ax);
        if (ay == 0) fc_piece(V, y, i, &py, &ay);
        u64 run = ax < ay ? ax : ay;
        run = run < m - i ? run : m - i;
        while (run > 0) {
            const u32 take = run < 8 * FC_ROUND ? (u32)run : 8u * FC_ROUND;
            u64 wa[FC_ROUND], wb[FC_ROUND];
#pragma unroll
            for (u32 q = 0; q < FC_ROUND; q++) {
                const u32 tq = take > 8 * q ? (take - 8 * q < 8 ? take - 8 * q : 8u) : 0u;
                wa[q] = tq ? load_be(V.suf, V.sufN, px + 8 * q, tq) : 0ull;
                wb[q] = tq ? load_be(V.suf, V.sufN, py + 8 * q, tq) : 0ull;
            }
#pragma unroll
            for (u32 q = 0; q < FC_ROUND; q++) {
                if (wa[q] != wb[q]) {
                    *lcp = i + 8 * q + (__clzll(wa[q] ^ wb[q]) >> 3);
                    return wa[q] < wb[q] ? -1 : 1;
                }
            }
            px += take;
            py += take;
            ax -= take;
            ay -= take;
            i += take;
            run -= take;
        }
    }
    *lcp = m;
    return lx < ly ? -1 : (lx > ly ? 1 : 0);
}

#define MG_PER 64  // outputs per thread
#define F_FIRST 0xFFFFFFFFu

struct MergeLevel {
    const u32 *G, *L, *F;  // element ids (FC positions), LCP with predecessor, first-LCP bound
    u32 *Go, *Lo, *Fo;
    const u64 *K;          // cached key: 7 bytes at the group depth + remaining length (capped at 8)
    u64 *Ko;
    const u32 *pg;         // per pair: group
    const u32 *Cg;         // per group: common prefix length of all its strings
    const u64 *PA0, *PA1, *PB1;  // per pair: run A = [PA0, PA1), run B = [PA1, PB1) in output space
    const u32 *tstart;           // first thread of each pair (npairs+1)
    u32 *pc;                     // per pair: lcp of the two runs' first strings
    u8 *pfirst;                  // per pair: 1 if run A's first string comes first
    u32 npairs;
    FcView V;
};

__device__ __forceinline__ u32 min3u(u32 a, u32 b, u32 c) { return min(a, min(b, c)); }

// Compare two elements of one group by their cached keys at the group depth C
// (bytes [C, C+7) and the remaining length, capped at 8).  Different keys
// decide alone: they order the two strings and give their LCP, whatever else
// is known about them.  Equal keys of strings that end inside the key are
// equal strings.  Otherwise the strings agree on [0, C+7), and `tie` compares
// them from there (or from a larger known common prefix): only then are the
// elements' ids and bounds needed, which lets callers read them lazily.
template <class Tie>
__device__ __forceinline__ int cmp_key(u64 kx, u64 ky, u32 C, u64 *lcp, Tie tie)
{
    if (kx != ky) {
        *lcp = key_lcp(kx, ky, C);
        return kx < ky ? -1 : 1;
    }
    const u32 cnt = (u32)(kx & 0xFF);
    if (cnt < 8) {
        *lcp = C + cnt;
        return 0;
    }
    return tie(lcp);
}

// The same for elements whose strings are known to agree on [0, bound).
__device__ __forceinline__ int cmp_elem(const FcView &V, u32 gx, u64 kx, u32 gy, u64 ky, u32 bound, u32 C,
                                        u64 *lcp)
{
    return cmp_key(kx, ky, C, lcp, [&](u64 *l) { return fc_cmp(V, gx, gy, bound > C + 7 ? bound : C + 7, l); });
}

#define MW_NT 256
// 5 outputs per thread: the LDS windows (MW_TILE + 2 entries of 20 bytes,
// 25.6 KB) and at most 85 VGPRs fit six workgroups per compute unit
#define MW_IPT 5
#define MW_TILE (MW_NT * MW_IPT)  // outputs per workgroup

// co-rank in global memory: number of A elements among the first d outputs
__device__ u32 corank_global(const MergeLevel &M, u64 A0, u32 na, u64 B0, u32 nb, u32 d, u32 c, u32 C)
{
    const u32 *GA = M.G + A0, *FA = M.F + A0, *GB = M.G + B0, *FB = M.F + B0;
    const u64 *KA = M.K + A0, *KB = M.K + B0;
    u32 xlo = d > nb ? d - nb : 0, xhi = d < na ? d : na;
    u64 tmp;
    while (xlo < xhi) {
        const u32 mid = (xlo + xhi) >> 1;
        const u32 y = d - mid - 1;
        // keys first: the ids and bounds are read only when the keys tie
        const int r = cmp_key(KA[mid], KB[y], C, &tmp, [&](u64 *l) {
            const u32 bd = min3u(FA[mid], c, FB[y]);
            return fc_cmp(M.V, GA[mid], GB[y], bd > C + 7 ? bd : C + 7, l);
        });
        if (r <= 0) xlo = mid + 1;
        else xhi = mid;
    }
    return xlo;
}

// Per output tile of one merge level: the LCP and order of its pair's two
// first strings (from the group depth on, with the cached keys; written by the
// pair's first tile) and the co-rank of the tile's first output, so that the
// merge kernel starts without a global search.
__global__ void k_merge_split(MergeLevel M, u32 nblocks, u32 *split)
{
    const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nblocks) return;
    u32 lo = 0, hi = M.npairs;
    while (hi - lo > 1) {
        u32 mid = (lo + hi) >> 1;
        if (M.tstart[mid] <= t) lo = mid;
        else hi = mid;
    }
    const u32 p = lo;
    const u64 A0 = M.PA0[p], A1 = M.PA1[p], B1 = M.PB1[p];
    const u32 na = (u32)(A1 - A0), nb = (u32)(B1 - A1);
    const u32 C = M.Cg[M.pg[p]];
    u32 c = 0;
    u8 fa = 1;
    if (na > 0 && nb > 0) {
        u64 l;
        const int r = cmp_elem(M.V, M.G[A0], M.K[A0], M.G[A1], M.K[A1], C, C, &l);
        c = (u32)l;
        fa = r <= 0 ? 1 : 0;
    } else if (na == 0) {
        fa = 0;
    }
    if (t == M.tstart[p]) {
        M.pc[p] = c;
        M.pfirst[p] = fa;
    }
    const u32 d0 = (t - M.tstart[p]) * MW_TILE;
    split[t] = d0 >= na + nb ? na : corank_global(M, A0, na, A1, nb, d0, c, C);
}

// The merge's results: per output, the source (run, position in run), the
// string id, the LCP with the previous output and the string length (src and
// len optional).  sb/sid: the non-empty runs' front-coded starts, ascending,
// and their run numbers.
struct MergeOut {
    const u64 *sb;
    const u32 *sid;
    u32 kne;
    const u32 *fc_id, *fc_len;
    u64 *src;
    u32 *id, *lcp, *len;
};

__device__ __forceinline__ void merge_emit(const MergeOut &O, u64 x, u32 g, u32 l)
{
    if (O.src) {
        u32 lo = 0, hi = O.kne;  // largest j with sb[j] <= g
        while (hi - lo > 1) {
            u32 mid = (lo + hi) >> 1;
            if (O.sb[mid] <= g) lo = mid;
            else hi = mid;
        }
        O.src[x] = ((u64)O.sid[lo] << 32) | (u64)(g - O.sb[lo]);
    }
    O.id[x] = O.fc_id[g];
    O.lcp[x] = l;
    if (O.len) O.len[x] = O.fc_len[g];
}

// One merge level, merge-path style: each workgroup produces MW_TILE outputs of
// one pair.  Its A and B windows (plus the element before each) are staged in
// LDS; every thread co-ranks its MW_IPT outputs inside the window and merges them
// with the LCP rule; outputs are written back through LDS.  The last level
// (LAST) writes the merge's results instead of the next level's elements.
template <bool LAST>
__global__ __launch_bounds__(MW_NT, 6) void k_merge_level(MergeLevel M, u32 nblocks, const u32 *split, MergeOut O)
{
    __shared__ u32 sG[MW_TILE + 2], sL[MW_TILE + 2], sF[MW_TILE + 2];
    __shared__ u64 sK[MW_TILE + 2];
    const u32 blk = blockIdx.x;
    if (blk >= nblocks) return;
    u32 lo = 0, hi = M.npairs;
    while (hi - lo > 1) {
        u32 mid = (lo + hi) >> 1;
        if (M.tstart[mid] <= blk) lo = mid;
        else hi = mid;
    }
    const u32 p = lo;
    const u64 A0 = M.PA0[p], A1 = M.PA1[p], B0 = A1, B1 = M.PB1[p];
    const u32 na = (u32)(A1 - A0), nb = (u32)(B1 - B0);
    const u32 tot = na + nb;
    const u32 d0 = (blk - M.tstart[p]) * MW_TILE;
    if (d0 >= tot) return;
    const u32 d1 = min(tot, d0 + MW_TILE);
    const u32 c = M.pc[p];
    const u32 C = M.Cg[M.pg[p]];
    const bool firstA = M.pfirst[p] != 0;
    const u32 a0 = split[blk];
    u32 a1 = (d1 == tot) ? na : split[blk + 1];
    // Keep the windows inside both runs even if the co-ranks are not monotone
    // (runs that violate the sortedness precondition): na >= a1 >= a0,
    // a1 - a0 <= d1 - d0, and d1 - a1 <= nb.
    {
        const u32 lo = max(a0, d1 > nb ? d1 - nb : 0u);
        const u32 hi = min(a0 + (d1 - d0), na);
        a1 = a1 < lo ? lo : (a1 > hi ? hi : a1);
    }
    const u32 b0 = d0 - a0, b1 = d1 - a1;
    const u32 wa = a1 - a0, wb = b1 - b0;
    // LDS layout: [pa | A window (wa) | pb | B window (wb)], pa/pb = element before the window
    const u32 baseA = 1, baseB = wa + 2;
    for (u32 i = threadIdx.x; i < wa + 1; i += MW_NT) {
        if (i == 0 && a0 == 0) continue;
        const u64 gi = A0 + a0 + i - 1;
        sG[i] = M.G[gi]; sL[i] = M.L[gi]; sF[i] = M.F[gi]; sK[i] = M.K[gi];
    }
    for (u32 i = threadIdx.x; i < wb + 1; i += MW_NT) {
        if (i == 0 && b0 == 0) continue;
        const u64 gi = B0 + b0 + i - 1;
        sG[baseB - 1 + i] = M.G[gi]; sL[baseB - 1 + i] = M.L[gi]; sF[baseB - 1 + i] = M.F[gi];
        sK[baseB - 1 + i] = M.K[gi];
    }
    __syncthreads();
    const FcView &V = M.V;
    const u32 dd = threadIdx.x * MW_IPT;  // local diagonal of this thread
    const u32 dw = d1 - d0;
    u32 oG[MW_IPT], oL[MW_IPT], oF[MW_IPT];
    u64 oK[MW_IPT];
    u32 cnt = 0;
    if (dd < dw) {
        cnt = min((u32)MW_IPT, dw - dd);
        u64 tmp;
        // co-rank inside the window (indices relative to a0 / b0).  Along the
        // diagonal the cached keys alone say "A first" up to some x1, "tie"
        // (equal keys of continuing strings) up to x2, then "B first"; both
        // bounds are found from the keys, and only [x1, x2) is searched with
        // string comparisons, so a wavefront compares strings once per
        // halving of its widest tie range instead of at every search step
        // where some lane's keys tie.
        u32 xlo = dd > wb ? dd - wb : 0, xhi = dd < wa ? dd : wa;
        auto key_side = [&](u32 x) -> int {  // -1: A first by the keys, 0: tie, 1: B first
            const u64 ka = sK[baseA + x], kb = sK[baseB + (dd - x - 1)];
            if (ka != kb) return ka < kb ? -1 : 1;
            return (ka & 0xFF) < 8 ? -1 : 0;  // equal strings ending in the key: A first
        };
        u32 x1lo = xlo, x1hi = xhi;
        while (x1lo < x1hi) {
            const u32 mid = (x1lo + x1hi) >> 1;
            if (key_side(mid) < 0) x1lo = mid + 1;
            else x1hi = mid;
        }
        // (no tie at x1: the range is empty, as it is wherever keys decide)
        u32 x2lo = x1lo, x2hi = (x1lo < xhi && key_side(x1lo) == 0) ? xhi : x1lo;
        while (x2lo < x2hi) {
            const u32 mid = (x2lo + x2hi) >> 1;
            if (key_side(mid) <= 0) x2lo = mid + 1;
            else x2hi = mid;
        }
        xlo = x1lo;
        xhi = x2lo;
        // (the LCPs of the last probes that moved each bound: the pairs on
        // both sides of the co-rank, used below)
        u64 lcp_lo = 0, lcp_hi = 0;
        bool moved_lo = false, moved_hi = false;
        while (xlo < xhi) {
            const u32 mid = (xlo + xhi) >> 1;
            const u32 ia = baseA + mid, ib = baseB + (dd - mid - 1);
            if (cmp_elem(V, sG[ia], sK[ia], sG[ib], sK[ib], min3u(sF[ia], c, sF[ib]), C, &tmp) <= 0) {
                xlo = mid + 1;
                lcp_lo = tmp;
                moved_lo = true;
            } else {
                xhi = mid;
                lcp_hi = tmp;
                moved_hi = true;
            }
        }
        u32 a = xlo, b = dd - xlo;  // relative to the window
        const u32 ga = a0 + a, gb = b0 + b;  // relative to the runs
        u32 ha = 0, hb = 0;
        if (d0 + dd > 0) {
            // The previous output is A[ga-1] or B[gb-1] (LDS slots pa / pb).
            // The LCPs across the co-rank, u = lcp(A[a-1], B[b]) and
            // w = lcp(B[b-1], A[a]), are those of the search's last probes,
            // or else the keys decide them (a pair outside the tie range);
            // with p = lcp(A[a-1], A[a]) and q = lcp(B[b-1], B[b]) they say
            // which predecessor is the larger: of two strings not above X,
            // the one sharing more with X is the larger.  Only when both
            // tests tie are the two predecessors compared.
            const u32 pa = baseA + a - 1, pb = baseB + b - 1;
            const bool hasA = a < wa, hasB = b < wb;
            auto pair_lcp = [&](u32 ix, u32 iy, bool rec, u64 l) -> u32 {
                if (rec) return (u32)l;
                u64 t;
                cmp_key(sK[ix], sK[iy], C, &t, [&](u64 *ll) { return fc_cmp(V, sG[ix], sG[iy], C + 7, ll); });
                return (u32)t;
            };
            const u32 w = (hasA && gb > 0) ? pair_lcp(baseA + a, pb, moved_hi && xhi == a, lcp_hi) : 0u;
            const u32 u = (hasB && ga > 0) ? pair_lcp(pa, baseB + b, moved_lo && xlo == a, lcp_lo) : 0u;
            const u32 p = hasA ? sL[baseA + a] : 0u, q = hasB ? sL[baseB + b] : 0u;
            bool lastA;
            if (ga == 0) {
                lastA = false;
            } else if (gb == 0) {
                lastA = true;
            } else {
                int dec = 0;
                u32 bnd = 0;
                if (hasA) {
                    if (p != w) dec = p > w ? 1 : -1;
                    bnd = p < w ? p : w;
                }
                if (dec == 0 && hasB) {
                    if (u != q) dec = u > q ? 1 : -1;
                    const u32 bq = u < q ? u : q;
                    bnd = bq > bnd ? bq : bnd;
                }
                lastA = dec != 0 ? dec > 0 : cmp_elem(V, sG[pa], sK[pa], sG[pb], sK[pb], bnd, C, &tmp) > 0;
            }
            ha = hasA ? (lastA ? p : w) : 0u;
            hb = hasB ? (lastA ? u : q) : 0u;
        }
#pragma unroll
        for (u32 k = 0; k < MW_IPT; k++) {
            if (k >= cnt) break;
            bool takeA;
            u32 outl;
            const u32 ia = baseA + a, ib = baseB + b;
            if (a >= wa) {
                takeA = false;
                outl = hb;
            } else if (b >= wb) {
                takeA = true;
                outl = ha;
            } else if (ha > hb) {
                takeA = true;
                outl = ha;
            } else if (ha < hb) {
                takeA = false;
                outl = hb;
            } else {
                const u32 bound = min3u(sF[ia], c, sF[ib]);
                const int r = cmp_elem(V, sG[ia], sK[ia], sG[ib], sK[ib], bound > ha ? bound : ha, C, &tmp);
                outl = ha;
                if (r <= 0) {
                    takeA = true;
                    hb = (u32)tmp;
                } else {
                    takeA = false;
                    ha = (u32)tmp;
                }
            }
            if (d0 + dd + k == 0) outl = 0;
            if (takeA) {
                oG[k] = sG[ia]; oL[k] = outl; oF[k] = firstA ? sF[ia] : min(c, sF[ia]); oK[k] = sK[ia];
                a++;
                if (a < wa) ha = sL[baseA + a];
            } else {
                oG[k] = sG[ib]; oL[k] = outl; oF[k] = firstA ? min(c, sF[ib]) : sF[ib]; oK[k] = sK[ib];
                b++;
                if (b < wb) hb = sL[baseB + b];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (u32 k = 0; k < MW_IPT; k++) {
        if (k < cnt) {
            sG[dd + k] = oG[k]; sL[dd + k] = oL[k];
            if (!LAST) { sF[dd + k] = oF[k]; sK[dd + k] = oK[k]; }
        }
    }
    __syncthreads();
    const u64 ob = A0 + d0;
    for (u32 i = threadIdx.x; i < dw; i += MW_NT) {
        if (LAST) merge_emit(O, ob + i, sG[i], sL[i]);
        else { M.Go[ob + i] = sG[i]; M.Lo[ob + i] = sL[i]; M.Fo[ob + i] = sF[i]; M.Ko[ob + i] = sK[i]; }
    }
}

#define RM_PARTS 32  // workgroups per run

// Minimum LCP-with-predecessor over each run except its first element, i.e.
// the LCP of the run's first and last strings: RM_PARTS workgroups per run
// (blockIdx.y = part), one atomic each.
__global__ __launch_bounds__(256) void k_run_min(const u64 *run_begin, const u64 *P, const u32 *e, u32 *runmin)
{
    __shared__ u32 wmin[4];
    const u32 r = blockIdx.x;
    const u64 b = run_begin[r], n = P[r + 1] - P[r];
    const u64 i0 = 1 + (n * blockIdx.y) / RM_PARTS, i1 = 1 + (n * (blockIdx.y + 1)) / RM_PARTS;
    u32 mn = 0xFFFFFFFFu;
    for (u64 i = i0 + threadIdx.x; i < i1 && i < n; i += 256) {
        const u32 v = e[b + i];
        mn = v < mn ? v : mn;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const u32 y = __shfl_xor(mn, o, 64);
        mn = y < mn ? y : mn;
    }
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32 m = wmin[0];
        for (int w = 1; w < 4; w++) m = wmin[w] < m ? wmin[w] : m;
        if (m != 0xFFFFFFFFu) atomicMin(&runmin[r], m);
    }
}

// Common prefix length of each group: every string of run r shares
// min(lcp(head of the group's first run, head of r), runmin[r]) bytes with the
// group's first head.
__global__ void k_group_depth(const u64 *run_begin, const u64 *P, const u32 *run_group, const u32 *rep, u32 k,
                              const u32 *runmin, FcView V, u32 *Cg)
{
    const u32 r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    if (P[r + 1] == P[r]) return;
    const u32 g = run_group[r];
    const u32 r0 = rep[g];
    u32 v = runmin[r];
    if (r0 != r) {
        u64 l;
        fc_cmp(V, (u32)run_begin[r0], (u32)run_begin[r], 0, &l);
        v = min(v, (u32)l);
    }
    atomicMin(&Cg[g], v);
}

// ---- per-element state of the merge by one segmented scan over the runs
//
// Output position x of run r is front-coded entry g = run_begin[r] + x - P[r]
// with LCP e_g to its predecessor (0 at the run start).  Its state is
//   G = g, L = e_g, F = min e over (start, x] (the LCP with the run head; all
//   ones at the start), K = bytes [C, C+7) of its string and min(d_g - C, 8),
// C = the group's common prefix.  F and K follow a scan with the operator
// (reset, m, p, v): F restarts at run starts and takes minima; the 7-byte
// window at C keeps its first p bytes from the predecessor's window
// (p = clamp(e_g - C, 0, 7)) and takes the rest, v, from the entry's literal.
struct MOp {
    u32 rp;  // bit 3: reset, bits 0..2: p
    u32 m;
    u64 v;
};

__device__ __forceinline__ MOp mop_id() { return MOp{7u, 0xFFFFFFFFu, 0ull}; }

// a, then b
__device__ __forceinline__ MOp mop_cat(MOp a, MOp b)
{
    const u32 pa = a.rp & 7u, pb = b.rp & 7u;
    const u64 keep = pb ? (~0ull << (64 - 8 * pb)) : 0ull;
    MOp r;
    r.rp = ((a.rp | b.rp) & 8u) | (pa < pb ? pa : pb);
    r.m = (b.rp & 8u) ? b.m : (a.m < b.m ? a.m : b.m);
    r.v = (a.v & keep) | (b.v & ~keep);
    return r;
}

__device__ __forceinline__ MOp mop_shfl_up(MOp a, u32 d)
{
    MOp r;
    r.rp = __shfl_up(a.rp, d, 64);
    r.m = __shfl_up(a.m, d, 64);
    r.v = __shfl_up(a.v, d, 64);
    return r;
}

__device__ __forceinline__ MOp mop_shfl(MOp a, u32 src)
{
    MOp r;
    r.rp = __shfl(a.rp, src, 64);
    r.m = __shfl(a.m, src, 64);
    r.v = __shfl(a.v, src, 64);
    return r;
}

struct MScan {
    const u64 *run_begin, *P;
    const u32 *run_group, *Cg;
    const u32 *bfirst;  // run of every scan block's first element
    u32 k, n_out;
    FcView V;
    u32 *ties;  // set to 1 if two adjacent strings of a run agree on [0, C+7)
};

// The run holding the positions being walked: its output range [pr, pr1),
// front-coded start and group depth, kept in registers.
struct RunCur {
    u32 r;
    u64 pr, pr1, rb;
    u32 C;
};

__device__ __forceinline__ RunCur run_cur(const MScan &S, u32 r)
{
    return RunCur{r, S.P[r], S.P[r + 1], S.run_begin[r], S.Cg[S.run_group[r]]};
}

// advance to the run containing x (x >= the current run's start)
__device__ __forceinline__ void run_seek(const MScan &S, RunCur &c, u64 x)
{
    while (c.pr1 <= x) {
        c.r++;
        c.pr = c.pr1;
        c.pr1 = S.P[c.r + 1];
        c.rb = S.run_begin[c.r];
        c.C = S.Cg[S.run_group[c.r]];
    }
}

__device__ __forceinline__ u32 run_of(const u64 *P, u32 k, u64 x)
{
    u32 lo = 0, hi = k;  // largest j with P[j] <= x
    while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (P[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// 7 elements per thread: the apply kernel's LDS operators take 28 KB; it runs
// four workgroups per compute unit, with the registers to keep its elements'
// entries and LCPs for the output pass without spilling
#define MS_PER 7
#define MS_ITEMS (256 * MS_PER)  // elements per workgroup

// This thread's elements x = x0 + 256 q + threadIdx.x (q < MS_PER; lanes on
// consecutive elements): entry g, run depth C and the in-range / run-start
// bits, from the block's first run and the cursor, which moves only at run
// bounds -- before any load of the elements' data is issued.
struct MElems {
    u32 g[MS_PER], C[MS_PER];
    u32 in, start;  // bit q
};

__device__ __forceinline__ void mscan_locate(const MScan &S, u64 x0, MElems &E)
{
    RunCur c = run_cur(S, S.bfirst[blockIdx.x]);
    E.in = E.start = 0;
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        const u64 x = x0 + q * 256 + threadIdx.x;
        E.g[q] = 0;  // (a valid entry to load from: the workgroup has elements)
        E.C[q] = 0;
        if (x < S.n_out) {
            run_seek(S, c, x);
            E.g[q] = (u32)(c.rb + (x - c.pr));
            E.C[q] = c.C;
            E.in |= 1u << q;
            if (x == c.pr) E.start |= 1u << q;
        }
    }
}

// The operators of this thread's elements (identity out of range) and their
// LCPs e[q]: the entries' LCPs, lengths and literal offsets are loaded for all
// elements first, then every element's window bytes, then combined.  An
// operator's low byte carries the element's length count min(d - C, 8), so
// that the inclusive operator at x is the element's cached key.
__device__ __forceinline__ void mscan_ops(const MScan &S, const MElems &E, MOp *o, u32 *e)
{
    u32 d[MS_PER];
    u64 so[MS_PER];
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        e[q] = S.V.e[E.g[q]];
        d[q] = S.V.d[E.g[q]];
        so[q] = S.V.suf_off[E.g[q]];
    }
    u32 p[MS_PER];
    Raw8 lit[MS_PER];
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        if ((E.start >> q) & 1) e[q] = 0;
        const u32 C = E.C[q];
        p[q] = e[q] > C ? (e[q] - C < 7 ? e[q] - C : 7u) : 0u;
        const u32 from = C + p[q];  // first window byte the entry's literal supplies (>= e)
        const u32 to = d[q] < C + 7 ? d[q] : C + 7;
        const bool want = ((E.in >> q) & 1) && p[q] < 7 && to > from;
        lit[q] = raw8_issue(S.V.suf, S.V.sufN, want ? so[q] + (from - e[q]) : 0ull, want ? to - from : 0u);
    }
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        const bool st = (E.start >> q) & 1;
        const u32 C = E.C[q];
        MOp r;
        r.rp = (st ? 8u : 0u) | p[q];
        r.m = st ? 0xFFFFFFFFu : e[q];
        r.v = (d[q] > C ? (d[q] - C < 8 ? d[q] - C : 8u) : 0u) |
              (__builtin_bswap64(raw8_le(S.V.suf, lit[q])) >> (8 * p[q]));
        o[q] = ((E.in >> q) & 1) ? r : mop_id();
    }
}

// Ordered reduction / exclusive scan of one operator per thread over a
// 256-thread workgroup.
__device__ __forceinline__ MOp block_mop_reduce(MOp a)
{
    __shared__ MOp wsum[4];
    const u32 lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (u32 d = 1; d < 64; d <<= 1) {
        const MOp y = mop_shfl_up(a, d);
        if (lane >= d) a = mop_cat(y, a);
    }
    if (lane == 63) wsum[wv] = a;
    __syncthreads();
    MOp t = wsum[0];
    for (u32 w = 1; w < 4; w++) t = mop_cat(t, wsum[w]);
    __syncthreads();
    return t;
}

__device__ __forceinline__ MOp block_mop_exclusive(MOp a, MOp carry)
{
    __shared__ MOp wsum[4];
    const u32 lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    MOp inc = a;
#pragma unroll
    for (u32 d = 1; d < 64; d <<= 1) {
        const MOp y = mop_shfl_up(inc, d);
        if (lane >= d) inc = mop_cat(y, inc);
    }
    if (lane == 63) wsum[wv] = inc;
    MOp ex = mop_shfl_up(inc, 1);
    if (lane == 0) ex = mop_id();
    __syncthreads();
    MOp pre = carry;
    for (u32 w = 0; w < wv; w++) pre = mop_cat(pre, wsum[w]);
    __syncthreads();
    return mop_cat(pre, ex);
}

// The run of every scan block's first element (the run r with P[r] <= x <
// P[r+1], x = j MS_ITEMS): each non-empty run writes it for the blocks that
// start inside it.
__global__ void k_block_runs(const u64 *P, u32 k, u32 nb, u32 *bfirst)
{
    const u32 r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    const u64 a = P[r], b = P[r + 1];
    for (u64 j = (a + MS_ITEMS - 1) / MS_ITEMS; j * MS_ITEMS < b && j < nb; j++) bfirst[j] = r;
}

// Phase 1: the operator of every MS_ITEMS-element block.  Its reset, p and m
// parts need only each element's e and d.  Of its window, byte k (k < 7) is
// the one written by the block's last element with p <= k (a later element
// with a larger p keeps it), and the count byte is the last element's, so at
// most eight literal bytes are read per block instead of every element's.
__global__ __launch_bounds__(256) void k_mscan_reduce(MScan S, MOp *blk)
{
    // per wavefront, per window byte k < 7 and the count (7): last supplier + 1, block-relative (0: none)
    __shared__ u32 s_wl[4][8];
    __shared__ u32 s_rp[MS_ITEMS], s_m[MS_ITEMS];
    const u64 x0 = (u64)blockIdx.x * MS_ITEMS;
    MElems E;
    mscan_locate(S, x0, E);
    u32 e[MS_PER];
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) e[q] = S.V.e[E.g[q]];
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        const u32 i = q * 256 + threadIdx.x;
        const bool st = (E.start >> q) & 1;
        const u32 ee = st ? 0u : e[q], C = E.C[q];
        const u32 p = ee > C ? (ee - C < 7 ? ee - C : 7u) : 0u;
        s_rp[i] = ((E.in >> q) & 1) ? ((st ? 8u : 0u) | p) : 0xFFu;  // (0xFF: out of range)
        s_m[i] = st ? 0xFFFFFFFFu : ee;
    }
    __syncthreads();
    // this thread's MS_PER consecutive elements, in order
    MOp t = mop_id();
    u32 lastk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        const u32 i = threadIdx.x * MS_PER + q;
        const u32 rp = s_rp[i];
        if (rp == 0xFFu) break;  // (out of range from here on)
        MOp o;
        o.rp = rp;
        o.m = s_m[i];
        o.v = 0;
        t = mop_cat(t, o);
        const u32 p = rp & 7u;
#pragma unroll
        for (u32 k = 0; k < 7; k++)
            if (p <= k) lastk[k] = i + 1;
        lastk[7] = i + 1;
    }
    // the last supplier of each byte is the highest lane that has one
    // (a thread's elements follow those of the lanes below it)
#pragma unroll
    for (u32 k = 0; k < 8; k++) {
        const u64 m = __ballot(lastk[k] != 0);
        const u32 v = m ? (u32)__shfl((int)lastk[k], 63 - __clzll(m), 64) : 0u;
        if ((threadIdx.x & 63) == 0) s_wl[threadIdx.x >> 6][k] = v;
    }
    t = block_mop_reduce(t);  // (reset, p, m); its window is filled below (its barriers complete s_wl)
    u32 last[8];
#pragma unroll
    for (u32 k = 0; k < 8; k++) last[k] = max(max(s_wl[0][k], s_wl[1][k]), max(s_wl[2][k], s_wl[3][k]));
    __shared__ u64 s_v[8];
    if (threadIdx.x < 8) s_v[threadIdx.x] = 0;
    __syncthreads();
    // byte k comes from element last[k] - 1; the thread holding that
    // element's entry loads it
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        const u32 j = q * 256 + threadIdx.x + 1;
        u32 ks = 0;
#pragma unroll
        for (u32 k = 0; k < 8; k++)
            if (last[k] == j) ks |= 1u << k;
        if (ks) {
            const u32 g = E.g[q], C = E.C[q];
            const u32 ee = ((E.start >> q) & 1) ? 0u : e[q];
            const u32 d = S.V.d[g];
            const u64 so = S.V.suf_off[g];
            if (ks & 0x80u) s_v[7] = d > C ? (d - C < 8 ? d - C : 8u) : 0u;  // the count byte
#pragma unroll
            for (u32 k = 0; k < 7; k++)  // byte at position C + k of the string (its literal starts at e <= C + k)
                if (((ks >> k) & 1) && C + k < d) s_v[k] = (u64)S.V.suf[so + (C + k - ee)] << (8 * (7 - k));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 v = 0;
#pragma unroll
        for (u32 k = 0; k < 8; k++) v |= s_v[k];
        t.v = v;
        blk[blockIdx.x] = t;
    }
}

// Phase 2: exclusive scan of the block operators (one workgroup of 1024:
// each thread composes a chunk, the chunk composites are scanned by
// wavefront shuffles and one pass over the 16 wavefront totals).
__global__ __launch_bounds__(1024) void k_mscan_top(MOp *blk, u32 nb)
{
    __shared__ MOp wtot[16];
    const u32 per = (nb + 1023) / 1024;
    const u32 c0 = threadIdx.x * per, c1 = (c0 + per < nb) ? c0 + per : nb;
    // (operators loaded eight at a time, ahead of the chain that combines them)
    MOp t = mop_id();
    for (u32 i = c0; i < c1; i += 8) {
        MOp v[8];
#pragma unroll
        for (u32 j = 0; j < 8; j++) v[j] = (i + j < c1) ? blk[i + j] : mop_id();
#pragma unroll
        for (u32 j = 0; j < 8; j++) t = mop_cat(t, v[j]);
    }
    const u32 lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    MOp inc = t;
#pragma unroll
    for (u32 d = 1; d < 64; d <<= 1) {
        const MOp y = mop_shfl_up(inc, d);
        if (lane >= d) inc = mop_cat(y, inc);
    }
    if (lane == 63) wtot[wv] = inc;
    MOp ex = mop_shfl_up(inc, 1);
    if (lane == 0) ex = mop_id();
    __syncthreads();
    MOp pre = mop_id();
    for (u32 w = 0; w < wv; w++) pre = mop_cat(pre, wtot[w]);
    pre = mop_cat(pre, ex);
    for (u32 i = c0; i < c1; i += 8) {
        MOp v[8];
#pragma unroll
        for (u32 j = 0; j < 8; j++) v[j] = (i + j < c1) ? blk[i + j] : mop_id();
#pragma unroll
        for (u32 j = 0; j < 8; j++) {
            if (i + j < c1) blk[i + j] = pre;
            pre = mop_cat(pre, v[j]);
        }
    }
}

// Phase 3: every element's inclusive operator -> G, L, F, K (written with
// consecutive lanes on consecutive elements).
__global__ __launch_bounds__(256, 4) void k_mscan_apply(MScan S, const MOp *blk, u32 *G, u32 *L, u32 *F, u64 *K)
{
    __shared__ MOp ops[MS_ITEMS];
    const u64 x0 = (u64)blockIdx.x * MS_ITEMS;
    MElems E;
    mscan_locate(S, x0, E);
    MOp o[MS_PER];
    u32 e[MS_PER];
    mscan_ops(S, E, o, e);
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) ops[q * 256 + threadIdx.x] = o[q];
    __syncthreads();
    MOp t = mop_id();
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) t = mop_cat(t, ops[threadIdx.x * MS_PER + q]);
    MOp st = block_mop_exclusive(t, blk[blockIdx.x]);
    // adjacent strings of a run that agree on their whole cached key
    bool tie = false;
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) tie |= ((E.in >> q) & 1) && e[q] >= E.C[q] + 7;
    if (__ballot(tie) && (threadIdx.x & 63) == 0) *S.ties = 1u;
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        const u32 i = threadIdx.x * MS_PER + q;
        st = mop_cat(st, ops[i]);
        ops[i].m = st.m;
        ops[i].v = st.v;
    }
    __syncthreads();
#pragma unroll
    for (u32 q = 0; q < MS_PER; q++) {
        const u32 i = q * 256 + threadIdx.x;
        const u64 x = x0 + i;
        if (!((E.in >> q) & 1)) break;
        G[x] = E.g[q];
        L[x] = e[q];
        F[x] = ops[i].m;
        K[x] = ops[i].v;
    }
}

// The results straight from the elements, where no merge level runs (every
// group holds at most one non-empty run).
__global__ void k_merge_out(const u32 *G, const u32 *L, u32 n_out, MergeOut O)
{
    const u32 x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_out) return;
    merge_emit(O, x, G[x], L[x]);
}

// Host-plan header: [0] check flag, [1] literal-buffer size, [2, 2+k) run
// begins, [2+k, 2+2k) run ends, then the group offsets as packed u32.
__global__ __launch_bounds__(256) void k_merge_header(const u64 *rb, const u64 *re, u32 k, const u32 *go,
                                                      u32 groups, const u32 *bad, const u64 *sufN, u64 *H)
{
    const u64 t = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        H[0] = bad ? *bad : 0u;
        H[1] = sufN ? *sufN : 0ull;
    }
    if (t < k) {
        H[2 + t] = rb[t];
        H[2 + k + t] = re[t];
    }
    if (t <= groups) ((u32 *)(H + 2 + 2 * (u64)k))[t] = go[t];
}

__global__ __launch_bounds__(256) void k_check_merge_runs(const u64 *rb, const u64 *re, u32 k, u64 n_fc,
                                                          const u32 *e, const u32 *d, u32 *bad)
{
    const u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) {
        if (re[i] < rb[i] || re[i] > n_fc) atomicOr(bad, 1u);
        else if (re[i] > rb[i] && e[rb[i]] != 0) atomicOr(bad, 2u);
    }
    if (i < n_fc) {
        if (e[i] > d[i]) atomicOr(bad, 4u);
        if (i > 0 && e[i] > d[i - 1]) atomicOr(bad, 4u);
    }
}

struct MergeWs {
    DecWs dec;
    u32 *G0, *G1, *L0, *L1, *F0, *F1, *pc, *tstart, *sid, *pg, *Cg, *rgroup, *rep, *split, *runmin, *bfirst, *ties;
    MOp *mblk;
    u8 *pfirst;
    u64 *PA0, *PA1, *PB1, *P, *sb, *K0, *K1;
};

#define MERGE_MAX_K 65536
// merge plan entries over all levels: <= 2k pairs plus one copy-through entry
// per group and level (<= 18 levels)
#define MERGE_PCAP(k) (20 * (size_t)(k) + 4)

static void merge_layout(u64 n_out, u64 n_fc, u64 k, MergeWs *w, WsArena *a, WsCounter *c)
{
    dec_layout(n_fc, &w->dec, a, c);
#define MT(field, T, cnt)                       \
    do {                                         \
        if (a) w->field = a->take<T>(cnt);       \
        else c->take<T>(cnt);                    \
    } while (0)
    MT(G0, u32, n_out); MT(G1, u32, n_out); MT(L0, u32, n_out); MT(L1, u32, n_out);
    MT(F0, u32, n_out); MT(F1, u32, n_out); MT(K0, u64, n_out); MT(K1, u64, n_out);
    // host-planned arrays, in two contiguous blocks (each uploaded in one copy)
    MT(P, u64, k + 2); MT(sb, u64, k + 2); MT(sid, u32, k + 2); MT(rgroup, u32, k + 2); MT(rep, u32, k + 2);
    MT(PA0, u64, MERGE_PCAP(k)); MT(PA1, u64, MERGE_PCAP(k)); MT(PB1, u64, MERGE_PCAP(k));
    MT(pg, u32, MERGE_PCAP(k)); MT(tstart, u32, MERGE_PCAP(k) + 64);
    MT(Cg, u32, k + 2); MT(pc, u32, MERGE_PCAP(k)); MT(pfirst, u8, MERGE_PCAP(k));
    MT(split, u32, n_out / MW_TILE + MERGE_PCAP(k) + 64);  // tiles of one level
    MT(runmin, u32, k + 2); MT(mblk, MOp, n_out / MS_ITEMS + 2); MT(bfirst, u32, n_out / MS_ITEMS + 2);
    MT(ties, u32, 4);
#undef MT
}

// Host arrays to device arrays that lie in one block in this order: staged in
// pinned memory at the same relative offsets and uploaded by one asynchronous
// copy (the staging buffer is reused once the copy has run).  Without pinned
// memory: one copy each, and a wait before the host arrays go away.
struct UpPart {
    void *dst;
    const void *src;
    size_t bytes;
};

static int upload_parts(const UpPart *parts, int np, hipStream_t st)
{
    u8 *base = (u8 *)parts[0].dst;
    const size_t span = (size_t)((u8 *)parts[np - 1].dst - base) + parts[np - 1].bytes;
    void *pin = ss_upload_take(span);
    if (!pin) {
        for (int q = 0; q < np; q++)
            if (parts[q].bytes) SS_HIP(hipMemcpyAsync(parts[q].dst, parts[q].src, parts[q].bytes,
                                                      hipMemcpyHostToDevice, st));
        SS_HIP(hipStreamSynchronize(st));
        return SS_OK;
    }
    for (int q = 0; q < np; q++)
        if (parts[q].bytes) memcpy((u8 *)pin + ((u8 *)parts[q].dst - base), parts[q].src, parts[q].bytes);
    const hipError_t e = hipMemcpyAsync(base, pin, span, hipMemcpyHostToDevice, st);
    ss_upload_release(pin, st);
    if (e != hipSuccess) {
        ss_set_error("plan upload failed: %s", hipGetErrorString(e));
        return SS_ERR_HIP;
    }
    return SS_OK;
}

extern "C" size_t ss_lcp_merge_workspace(uint64_t n_out, uint64_t n_fc, uint32_t k)
{
    WsCounter c;
    MergeWs w;
    merge_layout(n_out, n_fc, k, &w, nullptr, &c);
    return c.used;
}

extern "C" int ss_lcp_merge(uint32_t k, const uint64_t *run_begin, const uint64_t *run_end, uint32_t groups,
                            const uint32_t *group_off, uint64_t n_fc, const uint32_t *fc_lcp, const uint32_t *fc_len,
                            const uint32_t *fc_id, const uint64_t *suf_off, const uint8_t *suf, uint64_t *out_src,
                            uint32_t *out_id, uint32_t *out_lcp, uint32_t *out_len, uint64_t out_cap,
                            uint64_t *n_out_host, void *ws, size_t ws_bytes, void *stream)
{
    ss_clear_error();
    if (n_fc >= 0xFFFFFFFFull) { ss_set_error("n_fc too large"); return SS_ERR_TOO_LARGE; }
    if (k == 0 || k > MERGE_MAX_K || groups == 0 || groups > k || !run_begin || !run_end || !group_off) {
        ss_set_error("lcp_merge: bad arguments (1 <= k <= %d, 1 <= groups <= k)", MERGE_MAX_K);
        return SS_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    // The format check of the front-coded runs runs on the device before the
    // run bounds are known on the host, so that one read-back serves both.
    // Its flag lives in the decoding part of the workspace, whose placement
    // depends on n_fc only.
    WsArena a0(ws, ws_bytes);
    DecWs d0;
    dec_layout(n_fc, &d0, &a0, nullptr);
    if (a0.overflow || !ws) {
        ss_set_error("workspace too small for %llu front-coded entries", (unsigned long long)n_fc);
        return SS_ERR_WORKSPACE;
    }
    const bool have_fc = fc_lcp && fc_len && fc_id && suf_off;
    if (have_fc) {
        SS_HIP(hipMemsetAsync(d0.bad, 0, sizeof(u32), st));
        k_check_merge_runs<<<(unsigned)ceil_div((n_fc > k ? n_fc : k) + 1, 256), 256, 0, st>>>(
            run_begin, run_end, k, n_fc, fc_lcp, fc_len, d0.bad);
        SS_CHECK_LAUNCH();
    }
    // Everything the host plan needs, packed on the device into one staging
    // array (after the decoding part of the workspace; the merge arrays reuse
    // that space later) and brought back by one copy.
    std::vector<u64> rb(k), re(k);
    std::vector<u32> go(groups + 1);
    const u64 hdr = 2 + 2 * (u64)k + ((u64)groups + 2) / 2;
    u64 *stage = a0.take<u64>(hdr);
    std::vector<u64> H(hdr);
    if (stage) {
        const u64 nt = (u64)k > (u64)groups + 1 ? (u64)k : (u64)groups + 1;
        k_merge_header<<<(unsigned)ceil_div(nt, 256), 256, 0, st>>>(run_begin, run_end, k, group_off, groups,
                                                                    have_fc ? d0.bad : nullptr,
                                                                    have_fc ? suf_off + n_fc : nullptr, stage);
        SS_CHECK_LAUNCH();
        SS_TRY(ss_read_bytes(stage, H.data(), sizeof(u64) * hdr, st));
        memcpy(rb.data(), H.data() + 2, sizeof(u64) * k);
        memcpy(re.data(), H.data() + 2 + k, sizeof(u64) * k);
        memcpy(go.data(), H.data() + 2 + 2 * (u64)k, sizeof(u32) * (groups + 1));
    } else {
        H[0] = H[1] = 0;
        u32 b32 = 0;
        if (have_fc) {
            SS_HIP(hipMemcpyAsync(&b32, d0.bad, sizeof(u32), hipMemcpyDeviceToHost, st));
            SS_HIP(hipMemcpyAsync(&H[1], suf_off + n_fc, sizeof(u64), hipMemcpyDeviceToHost, st));
        }
        SS_HIP(hipMemcpyAsync(rb.data(), run_begin, sizeof(u64) * k, hipMemcpyDeviceToHost, st));
        SS_HIP(hipMemcpyAsync(re.data(), run_end, sizeof(u64) * k, hipMemcpyDeviceToHost, st));
        SS_HIP(hipMemcpyAsync(go.data(), group_off, sizeof(u32) * (groups + 1), hipMemcpyDeviceToHost, st));
        SS_HIP(hipStreamSynchronize(st));
        H[0] = b32;
    }
    const u32 bad = (u32)H[0];
    const u64 sufN = H[1];
    if (go[0] != 0 || go[groups] != k) {
        ss_set_error("group_off must start at 0 and end at k");
        return SS_ERR_INVALID_ARG;
    }
    std::vector<u64> P(k + 1, 0);
    for (u32 j = 0; j < k; j++) {
        if (re[j] < rb[j] || re[j] > n_fc) {
            ss_set_error("run %u = [%llu, %llu) is not inside the %llu front-coded entries", j,
                         (unsigned long long)rb[j], (unsigned long long)re[j], (unsigned long long)n_fc);
            return SS_ERR_INVALID_ARG;
        }
        P[j + 1] = P[j] + (re[j] - rb[j]);
    }
    for (u32 g = 0; g < groups; g++)
        if (go[g + 1] < go[g]) {
            ss_set_error("group_off must be non-decreasing");
            return SS_ERR_INVALID_ARG;
        }
    const u64 n_out = P[k];
    if (n_out_host) *n_out_host = n_out;
    if (n_out == 0) return SS_OK;
    if (n_out > out_cap) {
        ss_set_error("merge output has %llu entries, capacity %llu", (unsigned long long)n_out,
                     (unsigned long long)out_cap);
        return SS_ERR_CAPACITY;
    }
    if (!have_fc || !out_id || !out_lcp) {
        ss_set_error("lcp_merge: null array");
        return SS_ERR_INVALID_ARG;
    }
    if (bad) {
        ss_set_error("malformed front-coded runs (code %u): runs must start with e = 0 and e_i <= d_i, "
                     "e_i <= d_{i-1}", bad);
        return SS_ERR_INVALID_ARG;
    }
    // non-empty runs sorted by front-coded start, to map positions back to runs
    std::vector<u32> order;
    for (u32 j = 0; j < k; j++)
        if (re[j] > rb[j]) order.push_back(j);
    std::sort(order.begin(), order.end(), [&](u32 x, u32 y) { return rb[x] < rb[y]; });
    for (size_t t = 1; t < order.size(); t++)
        if (re[order[t - 1]] > rb[order[t]]) {
            ss_set_error("runs overlap");
            return SS_ERR_INVALID_ARG;
        }
    const u32 kne = (u32)order.size();
    std::vector<u64> sbv(kne);
    std::vector<u32> sidv(kne);
    for (u32 t = 0; t < kne; t++) { sbv[t] = rb[order[t]]; sidv[t] = order[t]; }

    WsArena a(ws, ws_bytes);
    MergeWs w;
    merge_layout(n_out, n_fc, k, &w, &a, nullptr);
    if (a.overflow) {
        ss_set_error("workspace too small: need %zu bytes", ss_lcp_merge_workspace(n_out, n_fc, k));
        return SS_ERR_WORKSPACE;
    }

    // Strings are compared without decoding them, along psv chains over the
    // whole front-coded array (built after the scan below).  Every comparison
    // of two elements past their cached keys starts at byte C+7 or later of
    // their group (the group depth compares run heads, whose e is 0), and a
    // chain walk for byte i starts only at an entry with e > i: none takes
    // place unless the scan finds adjacent strings of a run that share C+7
    // bytes, and the chains are built only then.
    k_fill_u32<<<1, 64, 0, st>>>(w.ties, 0u, 1);
    SS_CHECK_LAUNCH();
    const FcView V{fc_lcp, fc_len, w.dec.psv, suf_off, suf, sufN};
    // group of every run, first non-empty run of every group, group depths, keys
    std::vector<u32> rg(k), rep(groups, 0);
    for (u32 g = 0; g < groups; g++) {
        bool found = false;
        for (u32 j = go[g]; j < go[g + 1]; j++) {
            rg[j] = g;
            if (!found && re[j] > rb[j]) { rep[g] = j; found = true; }
        }
    }
    {
        const UpPart parts[] = {{w.P, P.data(), sizeof(u64) * (k + 1)},
                                {w.sb, sbv.data(), sizeof(u64) * kne},
                                {w.sid, sidv.data(), sizeof(u32) * kne},
                                {w.rgroup, rg.data(), sizeof(u32) * k},
                                {w.rep, rep.data(), sizeof(u32) * groups}};
        SS_TRY(upload_parts(parts, 5, st));
    }
    SS_HIP(hipMemsetAsync(w.Cg, 0xFF, sizeof(u32) * groups, st));
    SS_HIP(hipMemsetAsync(w.runmin, 0xFF, sizeof(u32) * k, st));
    k_run_min<<<dim3(k, RM_PARTS), 256, 0, st>>>(run_begin, w.P, fc_lcp, w.runmin);
    SS_CHECK_LAUNCH();
    k_group_depth<<<(unsigned)ceil_div(k, 64), 64, 0, st>>>(run_begin, w.P, w.rgroup, w.rep, k, w.runmin, V, w.Cg);
    SS_CHECK_LAUNCH();
    {
        // front-coded LCP, length, literal offset and up to 7 literal bytes in (twice), state out
        SS_PROF("k_mscan", st, (double)n_out * (2.0 * 24.0 + 20.0));
        const MScan S{run_begin, w.P, w.rgroup, w.Cg, w.bfirst, k, (u32)n_out, V, w.ties};
        const u32 nb = (u32)ceil_div(n_out, MS_ITEMS);
        k_block_runs<<<(unsigned)ceil_div(k, 256), 256, 0, st>>>(w.P, k, nb, w.bfirst);
        SS_CHECK_LAUNCH();
        k_mscan_reduce<<<nb, 256, 0, st>>>(S, w.mblk);
        SS_CHECK_LAUNCH();
        k_mscan_top<<<1, 1024, 0, st>>>(w.mblk, nb);
        SS_CHECK_LAUNCH();
        k_mscan_apply<<<nb, 256, 0, st>>>(S, w.mblk, w.G0, w.L0, w.F0, w.K0);
    }
    SS_CHECK_LAUNCH();
    SS_TRY(psv_build(fc_lcp, n_fc, w.dec.psv, w.dec.tree, w.dec.cmin, w.dec.far, w.dec.fcnt, st, w.ties));
    u32 *G = w.G0, *L = w.L0, *F = w.F0, *Go = w.G1, *Lo = w.L1, *Fo = w.F1;
    u64 *K = w.K0, *Ko = w.K1;
    std::vector<u32> pgv;
    // segments of the output space per group
    std::vector<std::vector<std::pair<u64, u64>>> segs(groups);
    for (u32 g = 0; g < groups; g++)
        for (u32 j = go[g]; j < go[g + 1]; j++) segs[g].push_back({P[j], P[j + 1]});
    std::vector<u64> pa0, pa1, pb1;
    std::vector<u32> ts;
    // plan every level on the host, upload the plan once, launch all levels
    struct LevelPlan { size_t off, ts_off; u32 npt; };
    std::vector<LevelPlan> plan;
    std::vector<u32> tsv;
    for (;;) {
        bool more = false;
        for (auto &sg : segs) more |= sg.size() > 1;
        if (!more) break;
        LevelPlan L0{pa0.size(), tsv.size(), 0};
        tsv.push_back(0);
        std::vector<std::vector<std::pair<u64, u64>>> nxt(groups);
        for (u32 g = 0; g < groups; g++) {
            auto &sg = segs[g];
            for (size_t m = 0; m < sg.size(); m += 2) {
                const u64 A0 = sg[m].first, A1 = sg[m].second;
                const u64 B1 = (m + 1 < sg.size()) ? sg[m + 1].second : A1;
                nxt[g].push_back({A0, B1});
                if (sg.size() == 1 && A1 == A0) continue;  // empty finished group: nothing to move
                // pairs, odd runs and finished groups (copied through to the other buffer)
                pa0.push_back(A0); pa1.push_back(A1); pb1.push_back(B1); pgv.push_back(g);
                const u64 sz = B1 - A0;
                tsv.push_back(tsv.back() + (u32)ceil_div(sz ? sz : 1, MW_TILE));
            }
        }
        L0.npt = (u32)(pa0.size() - L0.off);
        plan.push_back(L0);
        segs.swap(nxt);
    }
    const size_t npairs_all = pa0.size();
    if (npairs_all > MERGE_PCAP(k)) {
        ss_set_error("internal: merge plan exceeds its workspace");
        return SS_ERR_INVALID_ARG;
    }
    if (npairs_all) {
        const UpPart parts[] = {{w.PA0, pa0.data(), sizeof(u64) * npairs_all},
                                {w.PA1, pa1.data(), sizeof(u64) * npairs_all},
                                {w.PB1, pb1.data(), sizeof(u64) * npairs_all},
                                {w.pg, pgv.data(), sizeof(u32) * npairs_all},
                                {w.tstart, tsv.data(), sizeof(u32) * tsv.size()}};
        SS_TRY(upload_parts(parts, 5, st));
    }
    const MergeOut O{w.sb, w.sid, kne, fc_id, fc_len, out_src, out_id, out_lcp, out_len};
    for (size_t li = 0; li < plan.size(); li++) {
        const LevelPlan &lp = plan[li];
        const bool last = li + 1 == plan.size();
        MergeLevel M{G, L, F, Go, Lo, Fo, K, Ko, w.pg + lp.off, w.Cg, w.PA0 + lp.off, w.PA1 + lp.off,
                     w.PB1 + lp.off, w.tstart + lp.ts_off, w.pc + lp.off, w.pfirst + lp.off, lp.npt, V};
        const u32 nblk = tsv[lp.ts_off + lp.npt];
        if (nblk > 0) {
            k_merge_split<<<(unsigned)ceil_div(nblk, 64), 64, 0, st>>>(M, nblk, w.split);
            SS_CHECK_LAUNCH();
            if (last) {
                // id, LCP, bound and key in, the string id gathered; id and LCP out
                SS_PROF("k_merge_level", st, (double)n_out * 32.0);
                k_merge_level<true><<<nblk, MW_NT, 0, st>>>(M, nblk, w.split, O);
            } else {
                // every element's id, LCP, bound and key read once and written once
                SS_PROF("k_merge_level", st, (double)n_out * 40.0);
                k_merge_level<false><<<nblk, MW_NT, 0, st>>>(M, nblk, w.split, O);
            }
        }
        SS_CHECK_LAUNCH();
        std::swap(G, Go);
        std::swap(L, Lo);
        std::swap(F, Fo);
        std::swap(K, Ko);
    }
    if (plan.empty()) {
        k_merge_out<<<(unsigned)ceil_div(n_out, 256), 256, 0, st>>>(G, L, (u32)n_out, O);
        SS_CHECK_LAUNCH();
    }
    return SS_OK;
}
