// Error state, host read-back, tuning and device-wide exclusive scans.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

static thread_local char g_err[512];

void ss_set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void ss_clear_error() { g_err[0] = 0; }

extern "C" const char *ss_last_error(void) { return g_err; }
extern "C" int ss_version(void) { return 100; }

int g_small_max = 1024;
int g_tile = 4096;
int g_digit_bits = 8;
int g_dedup_mode = 0;
int g_dedup_logb = 0;

extern "C" int ss_set_tuning(int param, int value)
{
    if (param == SS_TUNE_SMALL_MAX) {
        if (value != 128 && value != 256 && value != 512 && value != 1024) {
            ss_set_error("SS_TUNE_SMALL_MAX must be 128, 256, 512 or 1024");
            return SS_ERR_INVALID_ARG;
        }
        int old = g_small_max;
        g_small_max = value;
        return old;
    }
    if (param == SS_TUNE_TILE) {
        if (value < 1024 || value > 16384 || (value & (value - 1))) {
            ss_set_error("SS_TUNE_TILE must be a power of two in [1024, 16384]");
            return SS_ERR_INVALID_ARG;
        }
        int old = g_tile;
        g_tile = value;
        return old;
    }
    if (param == SS_TUNE_DIGIT_BITS) {
        if (value != 8 && value != 11) {
            ss_set_error("SS_TUNE_DIGIT_BITS must be 8 or 11");
            return SS_ERR_INVALID_ARG;
        }
        int old = g_digit_bits;
        g_digit_bits = value;
        return old;
    }
    if (param == SS_TUNE_DEDUP) {
        if (value < 0 || value > 2) {
            ss_set_error("SS_TUNE_DEDUP must be 0, 1 or 2");
            return SS_ERR_INVALID_ARG;
        }
        int old = g_dedup_mode;
        g_dedup_mode = value;
        return old;
    }
    if (param == SS_TUNE_DEDUP_LOG_BUCKETS) {
        if (value < 0 || value > 14) {
            ss_set_error("SS_TUNE_DEDUP_LOG_BUCKETS must be 0..14");
            return SS_ERR_INVALID_ARG;
        }
        int old = g_dedup_logb;
        g_dedup_logb = value;
        return old;
    }
    ss_set_error("unknown tuning parameter %d", param);
    return SS_ERR_INVALID_ARG;
}

// Small read-backs go through pinned host buffers (a copy into pageable
// memory is staged by the runtime and costs a second round trip).  The
// buffers come from a pool that grows to the number of threads reading at
// once and lives as long as the process; a thread takes one per read.
namespace {
constexpr size_t PIN_BYTES = 65536;
std::mutex g_pin_mu;
std::vector<void *> g_pin_free;

void *pin_take()
{
    {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        if (!g_pin_free.empty()) {
            void *p = g_pin_free.back();
            g_pin_free.pop_back();
            return p;
        }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, PIN_BYTES, hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
}

void pin_give(void *p)
{
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.push_back(p);
}

int read_back(const void *dev, void *host, size_t bytes, hipStream_t s)
{
    void *p = bytes <= PIN_BYTES ? pin_take() : nullptr;
    if (!p) {
        SS_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
        SS_HIP(hipStreamSynchronize(s));
        return SS_OK;
    }
    hipError_t e = hipMemcpyAsync(p, dev, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) memcpy(host, p, bytes);
    pin_give(p);
    if (e != hipSuccess) {
        ss_set_error("HIP error %s in a read-back", hipGetErrorString(e));
        return SS_ERR_HIP;
    }
    return SS_OK;
}
}  // namespace

int ss_read_bytes(const void *dev, void *host, size_t bytes, hipStream_t s) { return read_back(dev, host, bytes, s); }

// Pinned staging for uploads that must not wait: a buffer is taken, filled,
// copied from asynchronously, and handed back with an event recorded after
// the copy; it is reused once that event has completed.
namespace {
struct UpBuf {
    void *p;
    size_t cap;
    hipEvent_t ev;
    bool busy, pending;
};
std::mutex g_up_mu;
std::vector<UpBuf> g_up;
}  // namespace

void *ss_upload_take(size_t bytes)
{
    std::lock_guard<std::mutex> lk(g_up_mu);
    for (auto &b : g_up) {
        if (b.busy || b.cap < bytes) continue;
        if (b.pending) {
            if (hipEventQuery(b.ev) != hipSuccess) continue;  // its last copy is still running
            b.pending = false;
        }
        b.busy = true;
        return b.p;
    }
    UpBuf b{nullptr, bytes > 65536 ? bytes : 65536, nullptr, true, false};
    if (hipHostMalloc(&b.p, b.cap, hipHostMallocDefault) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
        hipHostFree(b.p);
        return nullptr;
    }
    g_up.push_back(b);
    return b.p;
}

int ss_upload_release(void *p, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_up_mu);
    for (auto &b : g_up)
        if (b.p == p) {
            b.busy = false;
            b.pending = hipEventRecord(b.ev, s) == hipSuccess;
            if (!b.pending) {
                // no event: wait for the stream instead, then the buffer is free
                hipStreamSynchronize(s);
            }
            return SS_OK;
        }
    return SS_OK;
}

int ss_read_u32(const u32 *dev, u32 *host, int count, hipStream_t s)
{
    return read_back(dev, host, sizeof(u32) * (size_t)count, s);
}

int ss_read_u64(const u64 *dev, u64 *host, int count, hipStream_t s)
{
    return read_back(dev, host, sizeof(u64) * (size_t)count, s);
}

// ---------------------------------------------------------------- scans
//
// Arrays of up to SCAN_ONE_MAX items: one workgroup, one launch.  Longer ones
// take three phases: per-block sums, one-workgroup scan of the block sums,
// then a per-block scan that adds the block's offset.  Blocks hold SCAN_ITEMS
// items.

#define SCAN_NT 256
#define SCAN_PER 16
#define SCAN_ITEMS (SCAN_NT * SCAN_PER)
#define SCAN_ONE_MAX 16384  // arrays up to this length: one launch

template <class T>
__device__ __forceinline__ T wave_incl_scan(T x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a workgroup of NT threads.
template <class T, int NT>
__device__ __forceinline__ T block_excl_scan(T v, T *total)
{
    __shared__ T wsum[NT / 64 + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T s = 0;
        for (int w = 0; w < NT / 64; w++) {
            T t = wsum[w];
            wsum[w] = s;
            s += t;
        }
        wsum[NT / 64] = s;
    }
    __syncthreads();
    T r = x - v + wsum[wid];
    *total = wsum[NT / 64];
    __syncthreads();
    return r;
}

template <class T>
__global__ __launch_bounds__(SCAN_NT) void k_scan_reduce(const T *in, u64 n, T *sums)
{
    const u64 b0 = (u64)blockIdx.x * SCAN_ITEMS;
    T s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {
        u64 i = b0 + (u64)k * SCAN_NT + threadIdx.x;
        if (i < n) s += in[i];
    }
    T tot;
    block_excl_scan<T, SCAN_NT>(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(1024) void k_scan_single(T *sums, u64 nb)
{
    // each thread owns a contiguous chunk of the block sums
    const u64 per = (nb + 1023) / 1024;
    const u64 c0 = threadIdx.x * per, c1 = (c0 + per < nb) ? c0 + per : nb;
    T s = 0;
    for (u64 i = c0; i < c1; i++) s += sums[i];
    T tot;
    T pre = block_excl_scan<T, 1024>(s, &tot);
    for (u64 i = c0; i < c1; i++) {
        T v = sums[i];
        sums[i] = pre;
        pre += v;
    }
}

// Element (k, t) of a block is item b0 + k*SCAN_NT + t in global memory (so
// that loads and stores are coalesced) and slot tr(...) of the LDS buffer;
// each thread scans SCAN_PER consecutive items (blocked layout) from LDS.  One
// pad slot per SCAN_PER items keeps the blocked reads off a single bank.
__device__ __forceinline__ u32 scan_slot(u32 idx) { return idx + idx / SCAN_PER; }

template <class T>
__global__ __launch_bounds__(SCAN_NT) void k_scan_apply(const T *in, T *out, u64 n, const T *sums)
{
    __shared__ T buf[SCAN_ITEMS + SCAN_ITEMS / SCAN_PER];
    const u64 b0 = (u64)blockIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {  // striped, coalesced loads
        const u32 idx = (u32)k * SCAN_NT + threadIdx.x;
        const u64 i = b0 + idx;
        buf[scan_slot(idx)] = (i < n) ? in[i] : (T)0;
    }
    __syncthreads();
    T v[SCAN_PER];
    T s = 0;
    const u32 j0 = threadIdx.x * SCAN_PER;  // this thread's consecutive items
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {
        v[k] = buf[scan_slot(j0 + k)];
        s += v[k];
    }
    T tot;
    T pre = block_excl_scan<T, SCAN_NT>(s, &tot) + sums[blockIdx.x];  // (its barriers order the reads above)
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {
        buf[scan_slot(j0 + k)] = pre;
        pre += v[k];
    }
    // the last block's last thread holds the total (items past n count as 0)
    if (threadIdx.x == SCAN_NT - 1 && b0 + SCAN_ITEMS >= n) out[n] = pre;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {  // striped, coalesced stores
        const u32 idx = (u32)k * SCAN_NT + threadIdx.x;
        const u64 i = b0 + idx;
        if (i < n) out[i] = buf[scan_slot(idx)];
    }
}

template <class T> __global__ void k_zero_one(T *out) { out[0] = 0; }

// Short arrays in one launch: thread t owns a contiguous chunk; every thread
// reads its chunk before the block scan's barriers, so in == out is fine.
template <class T>
__global__ __launch_bounds__(1024) void k_scan_one(const T *in, T *out, u64 n)
{
    const u64 per = (n + 1023) / 1024;
    const u64 c0 = threadIdx.x * per, c1 = (c0 + per < n) ? c0 + per : n;
    T s = 0;
    for (u64 i = c0; i < c1; i++) s += in[i];
    T tot;
    T pre = block_excl_scan<T, 1024>(s, &tot);
    for (u64 i = c0; i < c1; i++) {
        const T v = in[i];
        out[i] = pre;
        pre += v;
    }
    if (threadIdx.x == 0) out[n] = tot;
}

template <class T> u64 ss_scan_scratch_elems(u64 n) { return ceil_div(n, SCAN_ITEMS) + 1; }

template <class T> int ss_scan_exclusive(const T *in, T *out, u64 n, T *scratch, hipStream_t s)
{
    if (n == 0) {
        k_zero_one<T><<<1, 1, 0, s>>>(out);
        SS_CHECK_LAUNCH();
        return SS_OK;
    }
    if (n <= SCAN_ONE_MAX) {
        k_scan_one<T><<<1, 1024, 0, s>>>(in, out, n);
        SS_CHECK_LAUNCH();
        return SS_OK;
    }
    const u64 nb = ceil_div(n, SCAN_ITEMS);
    k_scan_reduce<T><<<(unsigned)nb, SCAN_NT, 0, s>>>(in, n, scratch);
    SS_CHECK_LAUNCH();
    k_scan_single<T><<<1, 1024, 0, s>>>(scratch, nb);
    SS_CHECK_LAUNCH();
    k_scan_apply<T><<<(unsigned)nb, SCAN_NT, 0, s>>>(in, out, n, scratch);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

// Scans whose length is read on the device (n = *n_dev * mult), for launch
// sequences that must not read counts back (captured graphs).  A fixed grid
// of SCAN_DEV_G workgroups: workgroup b takes the contiguous range
// [b*per, (b+1)*per) with per = ceil(n / SCAN_DEV_G), sums it (phase 1), one
// workgroup scans the SCAN_DEV_G sums (phase 2), and every workgroup scans its
// range from its offset in chunks of SCAN_ITEMS (phase 3).
#define SCAN_DEV_G 1024

__device__ __forceinline__ u64 scan_dev_n(const u32 *n_dev, u32 mult) { return (u64)(*n_dev) * mult; }

template <class T>
__global__ __launch_bounds__(SCAN_NT) void k_scand_reduce(const T *in, const u32 *n_dev, u32 mult, T *part)
{
    const u64 n = scan_dev_n(n_dev, mult);
    const u64 per = (n + SCAN_DEV_G - 1) / SCAN_DEV_G;
    const u64 c0 = blockIdx.x * per, c1 = (c0 + per < n) ? c0 + per : n;
    T sacc = 0;
    for (u64 i = c0 + threadIdx.x; i < c1; i += SCAN_NT) sacc += in[i];
    T tot;
    (void)block_excl_scan<T, SCAN_NT>(sacc, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(SCAN_DEV_G) void k_scand_top(T *part, const u32 *n_dev, u32 mult, T *out)
{
    const T v = part[threadIdx.x];
    T tot;
    const T x = block_excl_scan<T, SCAN_DEV_G>(v, &tot);
    part[threadIdx.x] = x;
    if (threadIdx.x == 0) out[scan_dev_n(n_dev, mult)] = tot;
}

template <class T>
__global__ __launch_bounds__(SCAN_NT) void k_scand_apply(const T *in, T *out, const u32 *n_dev, u32 mult,
                                                         const T *part)
{
    const u64 n = scan_dev_n(n_dev, mult);
    const u64 per = (n + SCAN_DEV_G - 1) / SCAN_DEV_G;
    const u64 c0 = blockIdx.x * per, c1 = (c0 + per < n) ? c0 + per : n;
    T carry = part[blockIdx.x];
    for (u64 b = c0; b < c1; b += SCAN_ITEMS) {
        const u64 e = (b + SCAN_ITEMS < c1) ? b + SCAN_ITEMS : c1;
        // blocked: thread t takes SCAN_PER consecutive items
        const u64 t0 = b + (u64)threadIdx.x * SCAN_PER;
        T v[SCAN_PER];
        T sacc = 0;
#pragma unroll
        for (int q = 0; q < SCAN_PER; q++) {
            v[q] = (t0 + q < e) ? in[t0 + q] : (T)0;
            sacc += v[q];
        }
        T tot;
        T pre = block_excl_scan<T, SCAN_NT>(sacc, &tot) + carry;
#pragma unroll
        for (int q = 0; q < SCAN_PER; q++) {
            if (t0 + q < e) out[t0 + q] = pre;
            pre += v[q];
        }
        carry += tot;
        __syncthreads();  // (in may alias out: the next chunk's reads follow every write)
    }
}

template <class T> u64 ss_scan_dev_scratch_elems() { return SCAN_DEV_G; }

template <class T> int ss_scan_exclusive_dev(const T *in, T *out, const u32 *n_dev, u32 mult, T *scratch,
                                             hipStream_t s)
{
    k_scand_reduce<T><<<SCAN_DEV_G, SCAN_NT, 0, s>>>(in, n_dev, mult, scratch);
    SS_CHECK_LAUNCH();
    k_scand_top<T><<<1, SCAN_DEV_G, 0, s>>>(scratch, n_dev, mult, out);
    SS_CHECK_LAUNCH();
    k_scand_apply<T><<<SCAN_DEV_G, SCAN_NT, 0, s>>>(in, out, n_dev, mult, scratch);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

template u64 ss_scan_dev_scratch_elems<u32>();
template int ss_scan_exclusive_dev<u32>(const u32 *, u32 *, const u32 *, u32, u32 *, hipStream_t);

template u64 ss_scan_scratch_elems<u32>(u64);
template u64 ss_scan_scratch_elems<u64>(u64);
template int ss_scan_exclusive<u32>(const u32 *, u32 *, u64, u32 *, hipStream_t);
template int ss_scan_exclusive<u64>(const u64 *, u64 *, u64, u64 *, hipStream_t);

// ------------------------------------------------------------ profiling

bool g_prof_on = false;

namespace {
std::string g_prof_only;  // record only scopes of this name (empty: all)
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
// Events are reused across profiling windows (creating two per launch costs
// host time inside the timed region).  They only mark times on the device, so
// they carry no system-scope fence.
std::vector<hipEvent_t> g_ev_free;

void prof_clear()
{
    for (auto &r : g_prof) {
        g_ev_free.push_back(r.a);
        g_ev_free.push_back(r.b);
    }
    g_prof.clear();
}

hipEvent_t ev_take()
{
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_ev_free.empty()) {
            hipEvent_t e = g_ev_free.back();
            g_ev_free.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

void ev_give(hipEvent_t e)
{
    if (!e) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_ev_free.push_back(e);
}
}  // namespace

ProfScope::ProfScope(const char *n, hipStream_t s, double b) : name(n), st(s), bytes(b), a(nullptr), on(g_prof_on)
{
    if (!on) return;
    if (!g_prof_only.empty() && g_prof_only != n) {
        on = false;
        return;
    }
    a = ev_take();
    if (!a || hipEventRecord(a, st) != hipSuccess) {
        ev_give(a);
        on = false;
    }
}

ProfScope::~ProfScope()
{
    if (!on) return;
    hipEvent_t b = ev_take();
    if (!b || hipEventRecord(b, st) != hipSuccess) {
        ev_give(a);
        ev_give(b);
        return;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(ProfRec{name, a, b, bytes});
}

void ss_prof_add_bytes(const char *name, double bytes)
{
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (size_t i = g_prof.size(); i-- > 0;)
        if (g_prof[i].name == name) {
            g_prof[i].bytes += bytes;
            return;
        }
}

void ss_prof_drop_last(const char *name)
{
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (size_t i = g_prof.size(); i-- > 0;)
        if (g_prof[i].name == name) {
            g_ev_free.push_back(g_prof[i].a);
            g_ev_free.push_back(g_prof[i].b);
            g_prof.erase(g_prof.begin() + (long)i);
            return;
        }
}

extern "C" void ss_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear();
    g_prof_on = on != 0;
}

extern "C" void ss_profile_only(const char *name)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_only = name ? name : "";
}

extern "C" int ss_profile_query(const char *name, double *ms, double *bytes, uint32_t *launches)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double t = 0, by = 0;
    uint32_t cnt = 0;
    for (auto &r : g_prof) {
        if (r.name != name) continue;
        float e = 0;
        hipEventSynchronize(r.b);
        if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) continue;
        t += e;
        by += r.bytes;
        cnt++;
    }
    if (ms) *ms = t;
    if (bytes) *bytes = by;
    if (launches) *launches = cnt;
    return cnt ? SS_OK : SS_ERR_INVALID_ARG;
}

extern "C" size_t ss_profile_names(char *buf, size_t cap)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::vector<std::string> names;
    for (auto &r : g_prof) {
        bool seen = false;
        for (auto &x : names) seen |= (x == r.name);
        if (!seen) names.push_back(r.name);
    }
    std::string all;
    for (size_t i = 0; i < names.size(); i++) all += (i ? "," : "") + names[i];
    if (buf && cap) {
        size_t m = all.size() < cap - 1 ? all.size() : cap - 1;
        memcpy(buf, all.data(), m);
        buf[m] = 0;
    }
    return all.size();
}
