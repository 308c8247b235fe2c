// Shared helpers of the strsort HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <map>
#include <mutex>

#include "../../include/strsort.h"

typedef uint8_t u8;
typedef uint32_t u32;
typedef uint64_t u64;
typedef uint16_t u16;

// ----------------------------------------------------------------- errors

void ss_set_error(const char *fmt, ...);
void ss_clear_error();

#define SS_HIP(call)                                                            \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            ss_set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                         __FILE__, __LINE__);                                   \
            return SS_ERR_HIP;                                                  \
        }                                                                       \
    } while (0)

#define SS_CHECK_LAUNCH()                                                       \
    do {                                                                        \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess) {                                                 \
            ss_set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                   \
            return SS_ERR_HIP;                                                  \
        }                                                                       \
    } while (0)

// Workgroups of `kernel` (nt threads) that the current device holds at once.
// A grid-stride launch of at most this many runs as one wave of workgroups:
// with more, the last workgroups -- each owning many tiles -- run while most
// of the device waits for them.
template <class K>
static unsigned resident(K kernel, int nt)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, unsigned> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(dev, (const void *)kernel);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, nt, 0) != hipSuccess || per < 1 ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        (void)hipGetLastError();
        return 2048;  // (not cached: asked again next time)
    }
    const unsigned g = (unsigned)per * (unsigned)cus;
    cache[key] = g;
    return g;
}

#define SS_TRY(expr)                                                            \
    do {                                                                        \
        int rc_ = (expr);                                                       \
        if (rc_ != SS_OK) return rc_;                                           \
    } while (0)

static inline u64 ceil_div(u64 a, u64 b) { return (a + b - 1) / b; }
static inline u64 align_up(u64 a, u64 b) { return (a + b - 1) / b * b; }

// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct WsArena {
    u8 *base;
    size_t cap;
    size_t used;
    bool overflow;
    explicit WsArena(void *p, size_t c) : base((u8 *)p), cap(c), used(0), overflow(false) {}
    template <class T> T *take(u64 count) {
        size_t bytes = (size_t)align_up(count * sizeof(T) + 1, 256);
        if (used + bytes > cap) { overflow = true; return nullptr; }
        T *r = (T *)(base + used);
        used += bytes;
        return r;
    }
};
// Same layout computed without memory (for the *_workspace queries).
struct WsCounter {
    size_t used = 0;
    template <class T> void take(u64 count) { used += (size_t)align_up(count * sizeof(T) + 1, 256); }
};

// Host read-back of small device values (synchronises the stream).
int ss_read_u32(const u32 *dev, u32 *host, int count, hipStream_t s);
int ss_read_u64(const u64 *dev, u64 *host, int count, hipStream_t s);
int ss_read_bytes(const void *dev, void *host, size_t bytes, hipStream_t s);
// Pinned host staging for asynchronous uploads (NULL if none can be had);
// release after enqueueing the copies from it.
void *ss_upload_take(size_t bytes);
int ss_upload_release(void *p, hipStream_t s);

// Opt-in launch timing (ss_profile_enable): a scope records an event pair on
// the stream around the launch it encloses.
extern bool g_prof_on;
struct ProfScope {
    const char *name;
    hipStream_t st;
    double bytes;
    hipEvent_t a;
    bool on;
    ProfScope(const char *n, hipStream_t s, double b);
    ~ProfScope();
};
#define SS_PROF(name, stream, bytes) ProfScope ss_prof_scope_(name, stream, (double)(bytes))
// add bytes to the latest record of `name` (for counts known only after a read-back)
void ss_prof_add_bytes(const char *name, double bytes);
// forget the latest record of `name` (a launch that turned out to have no work)
void ss_prof_drop_last(const char *name);

// Tunables (set by ss_set_tuning).
extern int g_small_max;
extern int g_tile;
extern int g_digit_bits;  // radix digit width (8 or 11 bits)
extern int g_dedup_mode;  // duplicate detection: 0 global table, 1 buckets for long lists, 2 buckets
extern int g_dedup_logb;  // log2 of the bucket count (0: by the list length)

// ------------------------------------------------------ device-wide scans

// Exclusive prefix sum of in[0..n) into out[0..n], out[n] = total.  In-place
// (in == out) is allowed.  Scratch: ss_scan_scratch_elems(n) elements of T.
template <class T> u64 ss_scan_scratch_elems(u64 n);
template <class T> int ss_scan_exclusive(const T *in, T *out, u64 n, T *scratch, hipStream_t s);
// The same with the length read on the device, n = *n_dev * mult (a fixed
// launch shape, no read-back; for captured graphs).  out[n] = total.
// Scratch: ss_scan_dev_scratch_elems() elements of T.
template <class T> u64 ss_scan_dev_scratch_elems();
template <class T> int ss_scan_exclusive_dev(const T *in, T *out, const u32 *n_dev, u32 mult, T *scratch,
                                             hipStream_t s);

// ------------------------------------------------------------ byte loads

// The first `take` (0..8) bytes at bytes[a..] as a little-endian word
// (byte a -> bits 7..0), the rest zero.  Reads only inside [bytes, bytes + N):
// the two aligned 8-byte words around the bytes when both lie inside, byte
// loads otherwise.  Both words are loaded unconditionally (no branch between
// them, so several calls can have their loads in flight together), through a
// pointer derived from `bytes` so that they stay global-memory loads.
__device__ __forceinline__ u64 load_le(const u8 *__restrict__ bytes, u64 N, u64 a, u32 take)
{
    if (take == 0) return 0;
    const u8 *pb = bytes + a;
    const u32 sh = (u32)((uintptr_t)pb & 7);
    const uintptr_t base = (uintptr_t)pb - sh;
    u64 v;
    if (base >= (uintptr_t)bytes && base + 16 <= (uintptr_t)(bytes + N)) {
        const u64 *w = (const u64 *)(pb - sh);
        const u64 w0 = w[0], w1 = w[1];
        v = sh == 0 ? w0 : ((w0 >> (8 * sh)) | (w1 << (64 - 8 * sh)));
    } else {
        v = 0;
        for (u32 t = 0; t < take; t++) v |= (u64)bytes[a + t] << (8 * t);
    }
    if (take < 8) v &= (1ull << (8 * take)) - 1ull;
    return v;
}

// load_le in two halves, for callers that issue the loads of several words
// before combining any of them.
struct Raw8 {
    u64 w0, w1, a;
    u32 sh, take;
    bool ok;
};

__device__ __forceinline__ Raw8 raw8_issue(const u8 *__restrict__ bytes, u64 N, u64 a, u32 take)
{
    Raw8 r;
    r.a = a;
    r.take = take;
    const u8 *pb = bytes + a;
    r.sh = (u32)((uintptr_t)pb & 7);
    const uintptr_t base = (uintptr_t)pb - r.sh;
    r.ok = take > 0 && base >= (uintptr_t)bytes && base + 16 <= (uintptr_t)(bytes + N);
    r.w0 = r.w1 = 0;
    if (r.ok) {
        const u64 *w = (const u64 *)(pb - r.sh);
        r.w0 = w[0];
        r.w1 = w[1];
    }
    return r;
}

__device__ __forceinline__ u64 raw8_le(const u8 *__restrict__ bytes, const Raw8 &r)
{
    if (r.take == 0) return 0;
    u64 v;
    if (r.ok) {
        v = r.sh == 0 ? r.w0 : ((r.w0 >> (8 * r.sh)) | (r.w1 << (64 - 8 * r.sh)));
    } else {
        v = 0;
        for (u32 t = 0; t < r.take; t++) v |= (u64)bytes[r.a + t] << (8 * t);
    }
    if (r.take < 8) v &= (1ull << (8 * r.take)) - 1ull;
    return v;
}

// The same bytes packed big-endian into the top of a 64-bit word (byte a ->
// bits 63..56), the rest zero: integer order of such words is byte order.
__device__ __forceinline__ u64 load_be(const u8 *__restrict__ bytes, u64 N, u64 a, u32 take)
{
    return __builtin_bswap64(load_le(bytes, N, a, take));
}

// Radix key of a string at byte depth d: the next 7 bytes (zero-padded)
// big-endian in bits 63..8, and min(len - d, 8) in bits 7..0.  Comparing keys
// as unsigned integers orders strings by their bytes [d, d+7) with the
// shorter-is-smaller rule: a count below 8 marks a string ending inside the
// window, and equal data with count 8 means "equal so far, both continue".
__device__ __forceinline__ u64 make_key(const u8 *__restrict__ bytes, u64 N, u64 off, u64 len, u64 d)
{
    u64 rem = len > d ? len - d : 0;
    u32 take = rem < 7 ? (u32)rem : 7u;
    u64 data = load_be(bytes, N, off + d, take);
    u32 cnt = rem < 8 ? (u32)rem : 8u;
    return (data & ~0xFFull) | cnt;
}

// LCP of two strings whose keys at depth d differ (or are equal with count < 8):
// d + min(equal leading data bytes, count_a, count_b).
__device__ __forceinline__ u32 key_lcp(u64 ka, u64 kb, u32 d)
{
    u64 x = (ka ^ kb) >> 8;
    u32 eq = x ? (u32)(__clzll(x << 8) >> 3) : 7u;
    u32 ca = (u32)(ka & 0xFF), cb = (u32)(kb & 0xFF);
    u32 m = ca < cb ? ca : cb;
    return d + (eq < m ? eq : m);
}

// Full LCP of strings a (len la) and b (len lb) starting the comparison at
// byte `from` (both are known to agree on [0, from)).
__device__ __forceinline__ u64 str_lcp_from(const u8 *__restrict__ bytes, u64 N, u64 oa, u64 la,
                                            u64 ob, u64 lb, u64 from)
{
    u64 m = la < lb ? la : lb;
    u64 i = from;
    while (i < m) {
        u64 r = m - i;
        u32 take = r < 8 ? (u32)r : 8u;
        u64 wa = load_be(bytes, N, oa + i, take);
        u64 wb = load_be(bytes, N, ob + i, take);
        if (wa != wb) return i + (__clzll(wa ^ wb) >> 3);
        i += take;
    }
    return m;
}

// Three-way comparison of string a (bytes pa) against string b (bytes pb),
// both from possibly different buffers, starting at byte `from`.  Writes the
// LCP to *lcp_out.  Returns <0, 0, >0.
__device__ __forceinline__ int str_cmp_from(const u8 *__restrict__ ba, u64 Na, u64 oa, u64 la,
                                            const u8 *__restrict__ bb, u64 Nb, u64 ob, u64 lb,
                                            u64 from, u64 *lcp_out)
{
    u64 m = la < lb ? la : lb;
    u64 i = from;
    while (i < m) {
        u64 r = m - i;
        u32 take = r < 8 ? (u32)r : 8u;
        u64 wa = load_be(ba, Na, oa + i, take);
        u64 wb = load_be(bb, Nb, ob + i, take);
        if (wa != wb) {
            *lcp_out = i + (__clzll(wa ^ wb) >> 3);
            return wa < wb ? -1 : 1;
        }
        i += take;
    }
    *lcp_out = m;
    return la < lb ? -1 : (la > lb ? 1 : 0);
}

// Three-way comparison of strings a and b of one buffer by a whole wavefront:
// lane l holds bytes [512c + 8l, 512c + 8l + 8) of round c, so one round
// covers 512 bytes.  The lowest lane that sees a difference or the end of the
// shorter string decides.  Every lane gets the result and the LCP.  Must be
// called by all 64 lanes with the same arguments.
__device__ __forceinline__ int wave_str_cmp(const u8 *__restrict__ bytes, u64 N, u64 oa, u64 la, u64 ob,
                                            u64 lb, u64 *lcp_out)
{
    const u64 m = la < lb ? la : lb;
    const u32 lane = __lane_id();
    for (u64 c = 0;; c += 512) {
        const u64 q = c + 8ull * lane;
        const u32 take = q < m ? (m - q < 8 ? (u32)(m - q) : 8u) : 0u;
        const u64 wa = load_be(bytes, N, oa + q, take);
        const u64 wb = load_be(bytes, N, ob + q, take);
        const u64 stop = __ballot(wa != wb || take < 8);
        if (stop) {
            const int src = __ffsll((unsigned long long)stop) - 1;
            u64 l;
            int r;
            if (wa != wb) {
                l = q + (__clzll(wa ^ wb) >> 3);
                r = wa < wb ? -1 : 1;
            } else {
                l = q + take;
                r = la < lb ? -1 : (la > lb ? 1 : 0);
            }
            *lcp_out = __shfl(l, src);
            return __shfl(r, src);
        }
    }
}

// Binary search: number of entries of the sorted array a[0..n) that are <= x.
template <class T>
__device__ __forceinline__ u64 upper_bound_dev(const T *a, u64 n, T x)
{
    u64 lo = 0, hi = n;
    while (lo < hi) {
        u64 mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ u64 lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Wave-aggregated append: returns the slot for lanes with pred set.  Must be
// reached by the whole wavefront.
__device__ __forceinline__ u32 wave_append(bool pred, u32 *counter)
{
    u64 m = __ballot(pred);
    if (m == 0) return 0;
    u32 leader = __ffsll((unsigned long long)m) - 1;
    u32 base = 0;
    if (__lane_id() == leader) base = atomicAdd(counter, (u32)__popcll(m));
    base = __shfl(base, leader, 64);
    return base + (u32)__popcll(m & lanemask_lt());
}
