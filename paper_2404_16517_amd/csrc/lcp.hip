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
