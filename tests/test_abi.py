"""The C ABI library loads on a host without a GPU and exports every entry
point include/c2.h declares; host-only argument checks behave as documented.
No call here enqueues device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "c2.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:c2_status|size_t|const char \*)\s*(c2_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2010_11497_amd import c2
    if not os.path.exists(c2.LIB_PATH):
        from paper_2010_11497_amd import build
        build.build()
    return c2.load()


def test_header_lists_entry_points():
    names = declared()
    from paper_2010_11497_amd import c2
    assert names == sorted(c2.SYMBOLS)
    assert len(names) == 25


def test_library_exports_every_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_workspace_queries_host_only(lib):
    from paper_2010_11497_amd import c2
    p = c2.params(8, 1024, 2000, 30)
    n, m, nnz = 6000, 3700, 975556
    sizes = [lib.c2_workspace_bytes(n, m, nnz, ctypes.byref(p), op) for op in range(5)]
    assert all(s > 0 for s in sizes)
    # the build workspace holds the per-user partial lists
    assert sizes[c2.OP_BUILD] > 2 * 4 * n * 8 * 30
    bad = c2.params(8, 1024, 2000, 33)          # k > 32
    assert lib.c2_workspace_bytes(n, m, nnz, ctypes.byref(bad), c2.OP_BUILD) == 0
    assert b"k = 33" in lib.c2_last_error()
    assert lib.c2_workspace_bytes(n, 200000, nnz, ctypes.byref(p), c2.OP_BUILD) > 0    # DBLP-sized
    assert lib.c2_workspace_bytes(n, (1 << 19) + 1, nnz, ctypes.byref(p), c2.OP_BUILD) == 0
    assert b"m = 524289" in lib.c2_last_error()
    # the store takes what is left: the default holds more than the minimum
    assert (lib.c2_workspace_bytes(n, m, nnz, ctypes.byref(p), c2.OP_LOCAL_KNN) >
            lib.c2_workspace_bytes(n, m, nnz, ctypes.byref(p), c2.OP_LOCAL_KNN_MIN) > 0)
    assert lib.c2_workspace_bytes(n, m, nnz, ctypes.byref(p), 99) == 0
    fp = c2.params(1, 1024, 1, 1)                # fingerprint: p->b is the width in bits
    assert lib.c2_workspace_bytes(n, m, nnz, ctypes.byref(fp), c2.OP_FINGERPRINT) >= n * 128
    assert lib.c2_workspace_bytes(n, m, nnz, ctypes.byref(c2.params(1, 8193, 1, 1)),
                                  c2.OP_FINGERPRINT) == 0


def test_argument_errors_before_enqueue(lib):
    from paper_2010_11497_amd import c2
    P = c2.Profiles(10, 5, 20, 0, 0)
    p = c2.params(2, 4, 3, 2)
    assert lib.c2_build(ctypes.byref(P), None, ctypes.byref(p), 0, None, None, None, None, None, 0,
                        None) == -1
    assert lib.c2_hash_items(None, 1, 4, 5, None, None) == -1
    assert lib.c2_graph_create(ctypes.byref(P), None, ctypes.byref(p), None, None, None, None,
                               None, 0, None, None) == -1
    q = c2.Profiles(10, 5, 20, 1, 1)           # dummy non-null pointers; fails on params first
    bad = c2.params(0, 4, 3, 2)
    assert lib.c2_cluster(ctypes.byref(q), ctypes.c_void_p(1), ctypes.byref(bad), 0, None,
                          ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1),
                          ctypes.c_void_p(1), 1 << 30, None) == -1
    ok = c2.params(2, 4, 3, 2)
    assert lib.c2_cluster(ctypes.byref(q), ctypes.c_void_p(1), ctypes.byref(ok), 0, None,
                          ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1),
                          ctypes.c_void_p(1), 16, None) == -3      # workspace too small
    assert lib.c2_local_knn(ctypes.byref(q), ctypes.c_void_p(1), ctypes.c_void_p(1),
                            ctypes.c_void_p(1), ctypes.byref(ok), 7, None, ctypes.c_void_p(1),
                            ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 30, None) == -1  # form
    assert lib.c2_graph_destroy(None) == 0
    nnz = ctypes.c_uint64()
    for B in (0, 8193):                         # fingerprint width out of range
        assert lib.c2_fingerprint(ctypes.byref(q), ctypes.c_void_p(1), B, ctypes.c_void_p(1),
                                  ctypes.c_void_p(1), ctypes.byref(nnz), ctypes.c_void_p(1),
                                  1 << 30, None) == -1
    assert lib.c2_fingerprint(ctypes.byref(q), ctypes.c_void_p(1), 1024, ctypes.c_void_p(1),
                              ctypes.c_void_p(1), ctypes.byref(nnz), ctypes.c_void_p(1), 16,
                              None) == -3          # workspace too small


def test_training_entry_points_host_checks(lib):
    from paper_2010_11497_amd import c2
    assert lib.c2_assign_train_workspace_bytes(3, 1, 64) == 0          # odd batch
    assert b"nrows = 3" in lib.c2_last_error()
    assert lib.c2_assign_train_workspace_bytes(2, 1, 96) == 0          # b not a multiple of 64
    small = lib.c2_assign_train_workspace_bytes(2, 1, 64)
    big = lib.c2_assign_train_workspace_bytes(4096, 16, 8192)
    # the big batch holds its logits (fp32) and their gradient (bf16)
    assert small > 0 and big > 4096 * 16 * 8192 * 6
    one = ctypes.c_void_p(1)
    assert lib.c2_adam_step(one, one, one, one, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None, None) == -1
    assert lib.c2_adam_step(None, one, one, one, 10, 1e-3, 0.9, 0.999, 1e-8, 1, None, None) == -1
    assert lib.c2_adam_step(one, one, one, one, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None, None) == 0
    P = c2.Profiles(10, 5, 20, 1, 1)
    o = c2.TrainOpts(1.0, 1.0, 1.0)
    assert lib.c2_assign_train_grad(ctypes.byref(P), one, 4, one, one, one, one, one, 1, 64,
                                    ctypes.byref(o), one, one, one, one, one, one, one, 16,
                                    None) == -3            # workspace too small
