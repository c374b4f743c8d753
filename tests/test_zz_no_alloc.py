"""c2_build_noalloc (the build on the library's fixed per-GPU workspace, for
callers that cannot allocate) against c2_build with a caller workspace, through
the C ABI: bit-identical graphs on two calls in a row, the second on a smaller
input, in both forms; sizes beyond the fixed workspace are refused before any
device work."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2010_11497_amd import c2, synth  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_equals_build_two_calls():
    cases = [  # (seed, n, m, lo, hi, zipf, t, b, cap, k): the second is smaller
        (71, 3000, 1500, 5, 80, 1.0, 6, 64, 300, 16),
        (72, 700, 400, 2, 40, 0.8, 4, 16, 90, 10),
    ]
    for form in (c2.FORM_PLAIN, c2.FORM_BATCHED):
        for seed, n, m, lo, hi, zipf, t, b, cap, k in cases:
            say("noalloc form=%d seed=%d n=%d m=%d t=%d b=%d cap=%d k=%d"
                % (form, seed, n, m, t, b, cap, k))
            P = synth.random_profiles(seed, n, m, lo, hi, zipf)
            dP = c2.DeviceProfiles.from_synth(P)
            tab = c2.tables_to_device(synth.hash_tables(t, seed + 1000))
            p = c2.params(t, b, cap, k)
            tu = c2.tuning(split_rounds=16)
            want = c2.build(dP, tab, p, form, tu)
            status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
            got = c2.build_noalloc(dP, tab, p, form, tu, status=status)
            torch.cuda.synchronize()
            assert int(status.item()) == 0
            for g, w in zip(got, want):
                assert np.array_equal(c2.to_u32(g), c2.to_u32(w))


def test_noalloc_refuses_sizes_beyond_its_workspace():
    L = c2.load()
    p = c2.params(8, 4096, 2000, 30)
    P = c2.Profiles(70000, 10000, 9800000, 1, 1)    # dummy pointers: refused before use
    need = L.c2_workspace_bytes(P.n, P.m, P.nnz, ctypes.byref(p), c2.OP_BUILD)
    assert need > 256 << 20
    one = ctypes.c_void_p(1)
    st = L.c2_build_noalloc(ctypes.byref(P), one, ctypes.byref(p), c2.FORM_PLAIN, None, one, one,
                            one, None, None)
    assert st == -3
    assert b"fixed" in L.c2_last_error()
