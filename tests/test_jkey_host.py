"""The 32-bit selection key of the GPU local-KNN kernel, checked on the host.

The MFMA path of the local KNN ranks a row's candidates by
key(I, U) = floor(I * (2^32 - 1) / U) with the neighbour id below it, and
recovers I from the key and S = |P_u| + |P_v| when it writes the list
(exact Jaccard order, reading R2/R3; Section II-F).  The kernel computes both
in fp32 around the hardware reciprocal; tests/jkey_check.c restates the two
functions in C and compares them with exact integer arithmetic over every
(I, U) the kernel can see (profiles below 2^15 items), with the reciprocal
correctly rounded and 1 or 2 ulps off.  The order argument itself is checked
here with exact integers.  tests/filter_check.c does the same for the fp32
test that turns candidates away before any key is computed: it must pass
every candidate whose exact key reaches a full heap's root.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
M = (1 << 32) - 1


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("jkey") / "jkey_check")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off",
                           os.path.join(HERE, "jkey_check.c"), "-o", exe, "-lm"])
    return exe


@pytest.mark.parametrize("ulps,stride", [(1, 1), (2, 7)])
def test_key_and_recovery_exact(checker, ulps, stride):
    """Every pair (stride 1) or every 7th union size: the key equals the exact
    floor and the recovered I equals I, fused or unfused final add."""
    r = subprocess.run([checker, str(ulps), str(stride)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "key mismatches 0, I mismatches 0" in r.stdout


def key(I, U):
    return I * M // U


def test_key_order_is_jaccard_order():
    """Two different fractions with denominators below 2^16 differ by at least
    1/(b*d) > 1/(2^32 - 1), so their keys differ in the same direction; equal
    fractions have equal keys.  Checked on the closest pairs there are
    (neighbours in the Farey sequence of the largest denominators) and on
    equal fractions written with different denominators."""
    for a, b, c, d in [(1, 65535, 1, 65534), (65533, 65534, 65534, 65535),
                       (32767, 65535, 1, 2), (1, 2, 32767, 65533),
                       (32766, 65533, 1, 2), (0, 65535, 1, 65535)]:
        assert a * d < c * b
        assert key(a, b) < key(c, d), (a, b, c, d)
    for a, b, f in [(1, 2, 32767), (3, 7, 9362), (65534, 65534, 1), (0, 5, 13107)]:
        assert key(a, b) == key(a * f, b * f)


@pytest.fixture(scope="module")
def filter_checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("filter") / "filter_check")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off",
                           os.path.join(HERE, "filter_check.c"), "-o", exe, "-lm"])
    return exe


def test_filter_never_turns_away_a_candidate_that_enters(filter_checker):
    """The kernel's fp32 test against a full heap's root, with its margin
    (1 - 1e-6) and sigma from a reciprocal (or a quotient) up to 2 ulps off,
    passes the smallest intersection whose exact key reaches the root's, for
    640 root keys, every profile-length sum S below 2^16 and five splits of S;
    a padded column (+inf length) and an inactive row (NaN slope) fail it."""
    r = subprocess.run([filter_checker, "0.999999", "2", "1"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "turned away 0" in r.stdout


@pytest.mark.parametrize("margin", ["1.0", "0.9999999"])
def test_filter_check_sees_a_short_margin(filter_checker, margin):
    """Without the margin, or with one ten times shorter, rounding turns away
    candidates that would enter: the check above has something to find."""
    r = subprocess.run([filter_checker, margin, "0", "1"], capture_output=True, text=True)
    assert r.returncode == 1, r.stdout + r.stderr
    assert "turned away 0" not in r.stdout
