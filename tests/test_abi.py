"""Host-only checks of the C-ABI library: it loads without a GPU, exports every
entry point declared in include/strsort.h, and its argument checks fail
cleanly (these calls return before touching a device)."""
import ctypes
import os
import re

import pytest

import paper_2404_16517_amd as ss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "strsort.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ss_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    L = ss.lib()
    for n in names:
        assert hasattr(L, n), n


def test_version_and_error_text():
    assert ss.lib().ss_version() >= 100
    assert isinstance(ss.lib().ss_last_error(), bytes)


def test_workspace_queries_grow_with_n():
    L = ss.lib()
    for f in ("ss_sort_workspace", "ss_dist_prefix_workspace", "ss_partition_encode_workspace",
              "ss_fc_decode_workspace", "ss_gather_workspace"):
        a, b = getattr(L, f)(1000), getattr(L, f)(1_000_000)
        assert 0 < a < b, f
    assert L.ss_lcp_merge_workspace(1000, 10**6, 4) > L.ss_lcp_merge_workspace(1000, 1000, 4)


def test_argument_errors_without_device():
    L = ss.lib()
    P = ctypes.c_void_p
    # n beyond the 32-bit limit
    assert L.ss_sort(None, 0, None, 1 << 33, None, None, None, 0, None) == -3
    # null perm with n > 0
    assert L.ss_sort(None, 0, P(8), 10, None, None, None, 0, None) == -1
    assert b"null" in L.ss_last_error()
    # bad init_len / hash_bits
    assert L.ss_dist_prefix(None, 0, P(8), 10, 6, 64, P(8), None, None, 0, None) == -1
    assert L.ss_dist_prefix(None, 0, P(8), 10, 8, 4, P(8), None, None, 0, None) == -1
    # workspace too small is reported before any launch
    assert L.ss_dist_prefix(None, 0, P(8), 10, 8, 64, P(8), None, P(8), 16, None) == -2
    assert L.ss_sort(None, 0, P(8), 10, P(8), None, P(8), 16, None) == -2
    # select_splitters needs r >= 1 and n >= 1
    assert L.ss_select_splitters(0, P(8), 4, P(8), None) == -1
    # unknown batch flag; join needs k >= 1
    assert L.ss_sort_batch(P(8), 0, P(8), 10, P(8), 1, P(8), None, 4, P(8), 1 << 20, None) == -1
    assert L.ss_join_group_lcps(P(8), 0, P(8), P(8), 10, 0, P(8), P(8), 2, P(8), P(8), None) == -1
    assert L.ss_select_splitters_batch(P(8), 10, P(8), 0, 4, P(8), P(8), 256, None) == -1
    assert L.ss_select_splitters_batch(P(8), 10, P(8), 2, 4, P(8), P(8), 0, None) == -2
    # merge needs 1 <= k <= 65536
    assert L.ss_lcp_merge(0, P(8), P(8), 1, P(8), 1, P(8), P(8), P(8), P(8), P(8), P(8), P(8), P(8), None, 1,
                          None, None, 0, None) == -1
    assert L.ss_lcp_merge(4, P(8), P(8), 0, P(8), 1, P(8), P(8), P(8), P(8), P(8), P(8), P(8), P(8), None, 1,
                          None, None, 0, None) == -1
    # more groups than runs
    assert L.ss_lcp_merge(2, P(8), P(8), 3, P(8), 1, P(8), P(8), P(8), P(8), P(8), P(8), P(8), P(8), None, 1,
                          None, None, 0, None) == -1
    # the shared first read: a seed is required, the mode is 0..2; the seed's size is 256 + 16 n
    assert L.ss_dist_prefix_first_seed(P(8), 0, P(8), 10, None, 0, 8, 64, 0, None, P(8), 1 << 20, None) == -1
    assert L.ss_dist_prefix_first_seed(P(8), 0, P(8), 10, None, 0, 8, 64, 3, P(8), P(8), 1 << 20, None) == -1
    assert L.ss_dist_prefix_first_seed(P(8), 0, P(8), 10, P(8), 0, 8, 64, 0, P(8), P(8), 1 << 20, None) == -1
    assert L.ss_sort_seeded(P(8), 0, P(8), 10, None, P(8), None, P(8), 1 << 20, None) == -1
    assert L.ss_sort_batch_seeded(P(8), 0, P(8), 10, P(8), 1, None, P(8), None, 0, P(8), 1 << 20, None) == -1
    assert L.ss_sort_batch_seeded(P(8), 0, P(8), 10, P(8), 1, P(8), P(8), None, 2, P(8), 1 << 20, None) == -1
    assert L.ss_sort_seeded(P(8), 0, P(8), 1 << 33, P(8), P(8), None, P(8), 1 << 20, None) == -3
    assert L.ss_sort_seed_bytes(1000) == 256 + 16 * 1000


def test_tuning_validation():
    assert ss.set_tuning(ss.SS_TUNE_SMALL_MAX, 512) == 1024
    assert ss.set_tuning(ss.SS_TUNE_SMALL_MAX, 1024) == 512
    with pytest.raises(ss.StrsortError):
        ss.set_tuning(ss.SS_TUNE_SMALL_MAX, 300)
    with pytest.raises(ss.StrsortError):
        ss.set_tuning(ss.SS_TUNE_TILE, 3000)
    assert ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, 11) == 8
    assert ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, 8) == 11
    with pytest.raises(ss.StrsortError):
        ss.set_tuning(ss.SS_TUNE_DIGIT_BITS, 16)
    assert ss.set_tuning(ss.SS_TUNE_DEDUP, 1) == 0
    assert ss.set_tuning(ss.SS_TUNE_DEDUP, 0) == 1
    assert ss.set_tuning(ss.SS_TUNE_DEDUP_LOG_BUCKETS, 3) == 0
    assert ss.set_tuning(ss.SS_TUNE_DEDUP_LOG_BUCKETS, 0) == 3
    with pytest.raises(ss.StrsortError):
        ss.set_tuning(ss.SS_TUNE_DEDUP, 3)
    with pytest.raises(ss.StrsortError):
        ss.set_tuning(ss.SS_TUNE_DEDUP_LOG_BUCKETS, 15)


def test_device_batch_sort_and_graph_arguments():
    L = ss.lib()
    P = ctypes.c_void_p
    # status is required; rounds 1..1024; unknown flag bit
    assert L.ss_sort_batch_device(P(8), 0, P(8), 10, P(8), 1, P(8), None, 0, 4, None, P(8), 1 << 20, None) == -1
    assert L.ss_sort_batch_device(P(8), 0, P(8), 10, P(8), 1, P(8), None, 0, 0, P(8), P(8), 1 << 20, None) == -1
    assert L.ss_sort_batch_device(P(8), 0, P(8), 10, P(8), 1, P(8), None, 8, 4, P(8), P(8), 1 << 20, None) == -1
    # a round resolves at least 7 bytes: strings of L bytes need L // 7 + 2 rounds at most
    assert L.ss_sort_batch_device_rounds(256) == 38 and L.ss_sort_batch_device_rounds(0) == 2
    # capture needs a real stream; ending without a stream or output fails cleanly
    assert L.ss_graph_begin(None) == -1
    assert L.ss_graph_end(None, None) == -1
    assert L.ss_graph_launch(None, None) == -1
    L.ss_graph_destroy(None)
