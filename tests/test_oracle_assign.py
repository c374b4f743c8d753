"""Pins of the learned-assigner oracle (oracle/assign.py) against library
routines and closed forms; CPU only."""
import numpy as np
import pytest

from paper_2010_11497_amd import synth

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def A():
    from oracle import assign
    return assign


def test_bf16_round_matches_torch(A):
    rng = np.random.Generator(np.random.PCG64(1))
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-8, 8, 20000))).astype(np.float32)
    # exact ties: 1 + (2q+1) * 2^-8 sits halfway between two bf16 values
    ties = (1.0 + (2 * np.arange(64) + 1) * 2.0 ** -8).astype(np.float32)
    for v in (x, ties, -ties):
        want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(A.bf16_round(v.astype(np.float64)), want)
    assert A.bf16_round(1.0 + 2.0 ** -8) == 1.0                    # tie to even
    assert A.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6    # tie to even (up)


def test_embag_matches_torch_and_autograd(A):
    P = synth.random_profiles(2, 50, 40, 1, 9, 1.0)
    rng = np.random.Generator(np.random.PCG64(3))
    E = rng.standard_normal((P.m, 64))
    rows = np.array([3, 0, 49, 3, 17])
    got = A.embag(P.indptr, P.indices, E, rows)
    Et = torch.tensor(E, requires_grad=True)
    flat = torch.cat([torch.tensor(P.indices[P.indptr[u]:P.indptr[u + 1]].astype(np.int64))
                      for u in rows])
    lens = torch.tensor([P.indptr[u + 1] - P.indptr[u] for u in rows])
    offs = torch.cat([torch.zeros(1, dtype=torch.long), torch.cumsum(lens, 0)[:-1]])
    want = torch.nn.functional.embedding_bag(flat, Et, offs, mode="mean")
    assert np.allclose(got, want.detach().numpy(), rtol=1e-13, atol=1e-13)
    g = rng.standard_normal((len(rows), 64))
    (want * torch.tensor(g)).sum().backward()
    dE = A.embag_backward(P.indptr, P.indices, P.m, g, rows)
    assert np.allclose(dE, Et.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_hidden_identity_layer(A):
    """W1 = [I; 0], b1 = 0: the first 64 hidden units are ReLU(e_u), the rest 0;
    a single-item user's e_u is its E row exactly."""
    P = synth.profiles_from_sets([{5}, {1, 2}, {0, 1, 2, 3}], 8)
    E = A.bf16_round(np.random.Generator(np.random.PCG64(4)).standard_normal((8, 64)))
    W1 = np.zeros((256, 64))
    W1[:64] = np.eye(64)
    e, h = A.hidden(P.indptr, P.indices, E, W1, np.zeros(256))
    assert np.array_equal(e[0], E[5])
    assert np.array_equal(e[1], A.bf16_round((E[1] + E[2]) / 2))
    assert np.array_equal(h[:, :64], np.maximum(e, 0)) and not h[:, 64:].any()


def test_keys_closed_forms(A):
    """W2 rows one-hot on hidden unit c (b = 256) and b2 = 0: z = h, so the key
    is h's first maximum and the gap its top-two difference; all-equal logits
    give key 0 and gap 0."""
    rng = np.random.Generator(np.random.PCG64(5))
    h = np.floor(rng.uniform(0, 20, (30, 256)))          # many ties
    t, b = 2, 256
    W2 = np.vstack([np.eye(256)] * t)
    key, gap, _ = A.keys(h, W2, np.zeros(t * b), t, b)
    for u in range(30):
        row = list(h[u])
        assert key[0, u] == key[1, u] == row.index(max(row))
        s = sorted(row)
        assert gap[0, u] == s[-1] - s[-2]
    key, gap, _ = A.keys(h, np.zeros((t * b, 256)), np.zeros(t * b), t, b)
    assert not key.any() and not gap.any()


def test_weights_generator_is_seeded_bf16(A):
    E, W1, b1, W2, b2 = synth.assigner_weights(100, 2, 64, 7)
    assert E.dtype == np.uint16 and W2.shape == (128, 256) and b2.dtype == np.float32
    v = A.from_bf16_bits(W2)
    assert np.array_equal(A.bf16_round(v), v)
    assert np.array_equal(E, synth.assigner_weights(100, 2, 64, 7)[0])


def _tiny_training_case(seed, R=6, dim=3, hidden=5, t=2, b=4, m=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    P = synth.random_profiles(seed, 9, m, 1, 4, 0.0)
    rows = rng.integers(0, P.n, size=R)
    par = {"E": rng.standard_normal((m, dim)), "W1": rng.standard_normal((hidden, dim)),
           "b1": rng.standard_normal(hidden) * 0.3, "W2": rng.standard_normal((t * b, hidden)),
           "b2": rng.standard_normal(t * b) * 0.3}
    return P, rows, par, t, b, m


def _loss(A, P, rows, par, t, b, m, hyper):
    return A.train_forward_backward(P.indptr, P.indices, m, rows, par["E"], par["W1"], par["b1"],
                                    par["W2"], par["b2"], t, b, rounding=False, **hyper)


@pytest.mark.parametrize("seed", [11, 12, 13])
@pytest.mark.parametrize("hyper", [dict(w_neg=1.0, w_bal=1.0, w_ent=1.0),
                                   dict(w_neg=0.7, w_bal=3.0, w_ent=0.2)])
def test_training_gradients_match_finite_differences(A, seed, hyper):
    """Every gradient of the training objective (E, W1, b1, W2, b2) against
    central differences of the loss in float64, on a tiny batch of 3 pairs with
    small layers and the roundings switched off.  A wrong pairing of the
    non-neighbour (the roll direction), a dropped or mis-signed term of the
    loss or of the softmax/entropy derivative, or a transposed product fails
    here."""
    P, rows, par, t, b, m = _tiny_training_case(seed)
    loss, grads, inter = _loss(A, P, rows, par, t, b, m, hyper)
    assert np.abs(inter["pre"]).min() > 1e-3                 # away from the ReLU kink
    d = 1e-6
    for name in ("E", "W1", "b1", "W2", "b2"):
        x = par[name]
        fd = np.zeros_like(x)
        for idx in np.ndindex(x.shape):
            old = x[idx]
            x[idx] = old + d
            lp = _loss(A, P, rows, par, t, b, m, hyper)[0]["total"]
            x[idx] = old - d
            lm = _loss(A, P, rows, par, t, b, m, hyper)[0]["total"]
            x[idx] = old
            fd[idx] = (lp - lm) / (2 * d)
        got = grads["d" + name]
        assert np.allclose(got, fd, rtol=1e-5, atol=1e-8), name


def test_training_loss_closed_form_uniform(A):
    """All-zero output layer: every head is uniform (p = 1/b), so s = n = 1/b,
    q = 1/b, and the four parts are log b, -w_neg log(1 - 1/b), w_bal
    log(1 + 1e-12) (zero but for the logarithm's guard) and w_ent log b; the softmax's gradient sums to zero over each head."""
    P, rows, par, t, b, m = _tiny_training_case(21, b=8)
    par["W2"][:] = 0.0
    par["b2"][:] = 0.0
    hyper = dict(w_neg=0.5, w_bal=2.0, w_ent=0.25)
    loss, grads, inter = _loss(A, P, rows, par, t, b, m, hyper)
    assert loss["pos"] == pytest.approx(np.log(b), rel=1e-12)
    assert loss["neg"] == pytest.approx(-0.5 * np.log(1 - 1 / b), rel=1e-12)
    assert loss["bal"] == pytest.approx(2.0 * np.log1p(1e-12), rel=1e-6)    # the 1e-12 guard
    assert loss["ent"] == pytest.approx(0.25 * np.log(b), rel=1e-12)
    dz = inter["dz"].reshape(len(rows), t, b)
    assert np.abs(dz.sum(axis=-1)).max() < 1e-15


def test_adam_step_matches_torch(A):
    """Three Adam updates against torch.optim.Adam in float64 (same betas,
    eps and learning rate, bias correction from step 1)."""
    torch = pytest.importorskip("torch")
    rng = np.random.Generator(np.random.PCG64(31))
    x0 = rng.standard_normal(40)
    grads = [rng.standard_normal(40) for _ in range(3)]
    p = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    x, m1, m2 = x0.copy(), np.zeros(40), np.zeros(40)
    for step, g in enumerate(grads, start=1):
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        x, m1, m2 = A.adam_step(x, g, m1, m2, step, 3e-3)
        assert np.allclose(x, p.detach().numpy(), rtol=0, atol=1e-15)
