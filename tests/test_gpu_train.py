"""GPU parity of the assigner's training step (c2_assign_train_grad) and of the
Adam update (c2_adam_step) against the float64 oracle, through the C ABI.

The forward is made exact in the kernels' precision where a rounding would
decide a value (the bf16 embedding means and hidden layer): E holds small
integers and each W1 row adds two embedding dimensions, so e and h are the
oracle's bit for bit, while W2 and the biases are general.  The remaining
differences are then bounded by the arithmetic:
  * z: fp32 sums of exact bf16 products, |dz| error ~ 2^-16 |h||W2|;
  * dz is rounded to bf16 (relative 2^-9) before the products that read it,
    and dpre likewise before dW1 and de; fp32 sums add far less.
Each gradient is compared elementwise with a bound 2^-7 * (|A||B|) per
product (twice the bf16 step, which also covers the fp32 parts), propagated
through the chain with the oracle's own magnitudes.
"""
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


@pytest.fixture(scope="module")
def A():
    from oracle import assign
    return assign


def bf16_dev(bits):
    return torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16)


def f32(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def training_case(seed, n, m, t, b, B):
    """Profiles, a batch of B (user, neighbour) rows, and weights: E and W1 of
    synth.assigner_exact_weights and b1 in quarters from -4 to -2 (an exact
    forward, with about half of the hidden units cut by the ReLU), W2 and b2
    general."""
    P = synth.random_profiles(seed, n, m, 1, 40, 1.0)
    E, W1, _, _, _ = synth.assigner_exact_weights(m, t, b, seed + 1)
    _, _, _, W2, b2 = synth.assigner_weights(m, t, b, seed + 2)
    rng = np.random.Generator(np.random.PCG64(seed + 3))
    b1 = (-0.25 * rng.integers(8, 17, size=256)).astype(np.float32)
    rows = rng.integers(0, n, size=2 * B).astype(np.uint32)
    return P, rows, E, W1, b1, W2, b2


@pytest.mark.parametrize("seed,n,m,t,b,B", [(7100, 300, 90, 2, 64, 40),
                                            (7200, 3000, 700, 8, 256, 500),
                                            (7300, 5000, 2000, 4, 1024, 1200)])
def test_train_step_gradients(A, seed, n, m, t, b, B):
    say("train step", seed, n, m, t, b, B)
    P, rows, E, W1, b1, W2, b2 = training_case(seed, n, m, t, b, B)
    dP = c2.DeviceProfiles.from_synth(P)
    hyper = dict(w_neg=1.0, w_bal=1.5, w_ent=0.5)
    loss, dE, dW1, db1, dW2, db2 = c2.assign_train_grad(
        dP, torch.from_numpy(rows.view(np.int32)).cuda(), bf16_dev(E), bf16_dev(W1), f32(b1),
        bf16_dev(W2), f32(b2), t, b, **hyper)
    torch.cuda.synchronize()
    Ev, W1v, W2v = A.from_bf16_bits(E), A.from_bf16_bits(W1), A.from_bf16_bits(W2)
    wl, wg, it = A.train_forward_backward(P.indptr, P.indices, m, rows, Ev, W1v,
                                          b1.astype(np.float64), W2v, b2.astype(np.float64), t, b,
                                          **hyper)
    got = loss.cpu().numpy().astype(np.float64)
    want = np.array([wl["total"], wl["pos"], wl["neg"], wl["bal"], wl["ent"]])
    assert np.allclose(got, want, rtol=2e-4, atol=1e-5), (got, want)
    # bounds, built from the oracle's magnitudes
    u = 2.0 ** -7
    adz, ah, ae = np.abs(it["dz"]), np.abs(it["h"]), np.abs(it["e"])
    tol_dh = u * (adz @ np.abs(W2v)) + 1e-9
    tol_dpre = tol_dh * (it["pre"] > 0)
    adpre = np.abs(it["dpre"])
    tols = {"dW2": u * (adz.T @ ah) + 1e-9,
            "db2": u * adz.sum(axis=0) + 1e-9,
            "dW1": (tol_dpre + u * adpre).T @ ae + 1e-9,
            "db1": tol_dpre.sum(axis=0) + 1e-9,
            "dE": A.embag_backward(P.indptr, P.indices, m,
                                   (tol_dpre + u * adpre) @ np.abs(W1v), rows) + 1e-9}
    gots = {"dW2": dW2, "db2": db2, "dW1": dW1, "db1": db1, "dE": dE}
    for k, tol in tols.items():
        g = gots[k].cpu().numpy().astype(np.float64)
        err = np.abs(g - wg[k])
        assert np.all(err <= tol), (k, float((err / tol).max()))
        # and the comparison is not vacuous: the bound is small against the
        # values (looser along the W1 chain, whose sums cancel more)
        big = np.abs(wg[k]) > 1e-6
        limit = {"dW2": 0.02, "db2": 0.02, "dW1": 0.25, "db1": 0.25, "dE": 0.5}[k]
        assert np.median(tol[big] / np.abs(wg[k][big])) < limit, k
    assert 0.2 < (it["pre"] > 0).mean() < 0.8             # the ReLU mask matters


def test_train_step_dense_weights_close(A):
    """General (dense) W1 and E: the bf16 roundings of e and h may then differ
    from the oracle's in a few places, so the comparison is normwise."""
    P = synth.random_profiles(7400, 2000, 600, 1, 50, 1.0)
    t, b, B = 4, 256, 300
    E, W1, b1, W2, b2 = synth.assigner_weights(P.m, t, b, 7401)
    rows = np.random.Generator(np.random.PCG64(7402)).integers(0, P.n, 2 * B).astype(np.uint32)
    dP = c2.DeviceProfiles.from_synth(P)
    out = c2.assign_train_grad(dP, torch.from_numpy(rows.view(np.int32)).cuda(), bf16_dev(E),
                               bf16_dev(W1), f32(b1), bf16_dev(W2), f32(b2), t, b)
    torch.cuda.synchronize()
    wl, wg, _ = A.train_forward_backward(P.indptr, P.indices, P.m, rows, A.from_bf16_bits(E),
                                         A.from_bf16_bits(W1), b1.astype(np.float64),
                                         A.from_bf16_bits(W2), b2.astype(np.float64), t, b)
    assert abs(float(out[0][0]) - wl["total"]) <= 1e-3 * abs(wl["total"])
    for k, g in zip(("dE", "dW1", "db1", "dW2", "db2"), out[1:]):
        g = g.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(g - wg[k]) <= 0.02 * np.linalg.norm(wg[k]), k


def test_adam_step(A):
    """Three updates of 100,003 parameters against the float64 definition; the
    bf16 copy is the update rounded to nearest even."""
    rng = np.random.Generator(np.random.PCG64(7500))
    n = 100003
    x0 = rng.standard_normal(n).astype(np.float32)
    p, m1, m2 = f32(x0), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    p16 = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    x, a1, a2 = x0.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        g = (rng.standard_normal(n) * 10.0 ** rng.uniform(-4, 1, n)).astype(np.float32)
        c2.adam_step(p, f32(g), m1, m2, 3e-3, step, param_bf16=p16)
        x, a1, a2 = A.adam_step(x, g.astype(np.float64), a1, a2, step, 3e-3)
        torch.cuda.synchronize()
        got = p.cpu().numpy().astype(np.float64)
        # fp32 arithmetic on values of size |x| and a step of at most ~lr
        assert np.all(np.abs(got - x) <= 2e-6 * np.abs(x) + 3e-3 * 1e-4), step
    bits = p16.view(torch.int16).cpu().numpy().view(np.uint16)
    u = p.cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal(bits, ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16))


def test_training_lowers_the_loss():
    """A few hundred steps of learned.train on a small workload lower the
    objective and leave finite weights."""
    from paper_2010_11497_amd import learned
    P = synth.make_profiles(synth.WORKLOADS["n2k_m1k"])
    dP = c2.DeviceProfiles.from_synth(P)
    pairs = learned.exact_pairs(P, 2000, 10, seed=1)
    Asg = learned.Assigner(P.m, 4, 64, seed=3)
    st = learned.train(Asg, dP, pairs, steps=300, batch=256, w_bal=1.0)
    assert st.last_loss < st.first_loss
    for v in Asg.master.values():
        assert torch.isfinite(v).all()
