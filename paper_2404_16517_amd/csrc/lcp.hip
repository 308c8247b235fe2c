// LCP array of a given order and exact distinguishing prefixes (Section 2).
#include "common.hpp"

__global__ __launch_bounds__(256) void k_lcp(const u8 *bytes, u64 N, const u64 *off, u32 n,
                                             const u32 *perm, u32 *lcp)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0) {
        lcp[0] = 0;
        return;
    }
    const u32 a = perm[i - 1], b = perm[i];
    const u64 oa = off[a], la = off[a + 1] - oa;
    const u64 ob = off[b], lb = off[b + 1] - ob;
    lcp[i] = (u32)str_lcp_from(bytes, N, oa, la, ob, lb, 0);
}

// Wave-wide sum of a 64-bit value (every lane gets it).
__device__ __forceinline__ u64 wave_sum_u64(u64 v)
{
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// One wavefront per group g >= 1: the group's first output position G is the
// total size of the runs of groups before it; if the group is not empty and
// G > 0, lcp[G] becomes the LCP of the strings at output positions G-1 and G.
__global__ __launch_bounds__(256) void k_join_groups(const u8 *bytes, u64 N, const u64 *off, const u32 *order,
                                                     u64 n_out, u32 k, const u64 *rb, const u64 *re,
                                                     u32 groups, const u32 *go, u32 *lcp)
{
    const u32 g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const u32 lane = threadIdx.x & 63;
    if (g == 0 || g >= groups) return;  // uniform over the wavefront
    const u32 r1 = go[g + 1] < k ? go[g + 1] : k;
    const u32 r0 = go[g] < r1 ? go[g] : r1;
    u64 before = 0, own = 0;
    for (u32 r = lane; r < r1; r += 64) {
        const u64 sz = re[r] - rb[r];
        if (r < r0) before += sz;
        else own += sz;
    }
    before = wave_sum_u64(before);
    own = wave_sum_u64(own);
    if (own == 0 || before == 0 || before >= n_out) return;
    const u32 a = order[before - 1], b = order[before];
    const u64 oa = off[a], ob = off[b];
    u64 l;
    wave_str_cmp(bytes, N, oa, off[a + 1] - oa, ob, off[b + 1] - ob, &l);
    if (lane == 0) lcp[before] = (u32)l;
}

extern "C" int ss_join_group_lcps(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, const uint32_t *order,
                                  uint64_t n_out, uint32_t k, const uint64_t *run_begin, const uint64_t *run_end,
                                  uint32_t groups, const uint32_t *group_off, uint32_t *lcp, void *stream)
{
    ss_clear_error();
    if (groups == 0 || k == 0 || !offsets || !run_begin || !run_end || !group_off || (n_out > 0 && (!order || !lcp))) {
        ss_set_error("join_group_lcps needs groups >= 1, k >= 1 and non-null arrays");
        return SS_ERR_INVALID_ARG;
    }
    if (groups < 2 || n_out == 0) return SS_OK;
    hipStream_t st = (hipStream_t)stream;
    k_join_groups<<<(unsigned)ceil_div(groups, 4), 256, 0, st>>>(bytes, N, offsets, order, n_out, k, run_begin,
                                                                 run_end, groups, group_off, lcp);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

// dist of the string at sorted position i = min(len, 1 + max(lcp[i], lcp[i+1])),
// lcp[n] := 0; written at its input index.
__global__ __launch_bounds__(256) void k_dist_exact(const u64 *off, u32 n, const u32 *perm,
                                                    const u32 *lcp, u32 *dist)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32 a = lcp[i];
    const u32 b = (i + 1 < n) ? lcp[i + 1] : 0u;
    const u32 p = perm[i];
    const u64 len = off[p + 1] - off[p];
    const u64 m = (u64)(a > b ? a : b) + 1;
    dist[p] = (u32)(m < len ? m : len);
}

extern "C" int ss_lcp(const uint8_t *bytes, uint64_t N, const uint64_t *offsets, uint64_t n,
                      const uint32_t *perm, uint32_t *lcp, void *stream)
{
    ss_clear_error();
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (n == 0) return SS_OK;
    if (!offsets || !perm || !lcp) { ss_set_error("null pointer"); return SS_ERR_INVALID_ARG; }
    hipStream_t st = (hipStream_t)stream;
    k_lcp<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(bytes, N, offsets, (u32)n, perm, lcp);
    SS_CHECK_LAUNCH();
    return SS_OK;
}

// dist from a bound d with dist <= d <= len: min(d, 1 + max(lcp[i], lcp[i+1])).
__global__ __launch_bounds__(256) void k_dist_bounded(u32 n, const u32 *perm, const u32 *lcp, const u32 *d,
                                                      u32 *dist)
{
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32 a = lcp[i];
    const u32 b = (i + 1 < n) ? lcp[i + 1] : 0u;
    const u64 m = (u64)(a > b ? a : b) + 1;
    const u32 di = d[i];
    dist[perm ? perm[i] : i] = (u32)(m < di ? m : di);
}

extern "C" int ss_dist_exact_bounded(const uint32_t *perm, const uint32_t *lcp, const uint32_t *d, uint64_t n,
                                     uint32_t *dist, void *stream)
{
    ss_clear_error();
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (n == 0) return SS_OK;
    if (!lcp || !d || !dist) { ss_set_error("null pointer"); return SS_ERR_INVALID_ARG; }
    hipStream_t st = (hipStream_t)stream;
    {
        SS_PROF("k_dist_exact", st, (double)n * (perm ? 16.0 : 12.0));  // perm, lcp, d in; dist out
        k_dist_bounded<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>((u32)n, perm, lcp, d, dist);
    }
    SS_CHECK_LAUNCH();
    return SS_OK;
}

extern "C" int ss_dist_exact(const uint64_t *offsets, uint64_t n, const uint32_t *perm,
                             const uint32_t *lcp, uint32_t *dist, void *stream)
{
    ss_clear_error();
    if (n >= 0xFFFFFFFFull) { ss_set_error("n too large"); return SS_ERR_TOO_LARGE; }
    if (n == 0) return SS_OK;
    if (!offsets || !perm || !lcp || !dist) { ss_set_error("null pointer"); return SS_ERR_INVALID_ARG; }
    hipStream_t st = (hipStream_t)stream;
    {
        SS_PROF("k_dist_exact", st, (double)n * 28.0);  // perm, lcp, offsets in; dist out
        k_dist_exact<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(offsets, (u32)n, perm, lcp, dist);
    }
    SS_CHECK_LAUNCH();
    return SS_OK;
}
