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
