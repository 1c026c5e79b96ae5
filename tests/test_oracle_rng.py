"""Pins of the oracle's random numbers (SplitMix64 counter form, distinct draws, signs)."""
import numpy as np
from scipy import stats

from conftest import read_golden


def test_splitmix64_published_vector(orc):
    # Stream 0 of the counter form is the plain SplitMix64 sequence.
    want = [int(r[0]) for r in read_golden("splitmix64_seed1234567.txt")]
    got = [orc.rng_u64(1234567, 0, i) for i in range(len(want))]
    assert got == want


def test_streams_are_counter_offsets(orc):
    # stream s, index i is index s*2^40 + i of stream 0
    for s in (1, 2, 5):
        for i in (0, 7, 123456):
            assert orc.rng_u64(99, s, i) == orc.rng_u64(99, 0, (s << 40) + i)


def test_draw_distinct_basic(orc):
    for n, k in ((10, 10), (512, 10), (20000, 100), (3, 2), (1, 1)):
        out = orc.draw_distinct(2001, 0, n, k)
        assert len(set(out.tolist())) == k
        assert out.min() >= 0 and out.max() < n
    perm = orc.draw_distinct(7, 0, 50, 50)
    assert sorted(perm.tolist()) == list(range(50))


def test_draw_distinct_first_draw_is_uniform(orc):
    # n = 7 does not divide 2^64, so a missing rejection step or a wrong
    # modulus would bias the residues; chi-square over 14000 seeds.
    n = 7
    first = np.array([orc.draw_distinct(s, 0, n, 1)[0] for s in range(14000)])
    counts = np.bincount(first, minlength=n)
    assert stats.chisquare(counts).pvalue > 1e-4


def test_draw_distinct_matches_rejection_rule_small(orc):
    # n = 2^62 + 1: a quarter of all 64-bit words are rejected, so the
    # draw must skip them; values below the limit map by plain modulo.
    n = (1 << 62) + 1
    lim = (1 << 64) - ((1 << 64) % n)
    seq = [orc.rng_u64(5, 0, i) for i in range(64)]
    accepted = [u % n for u in seq if u < lim]
    got = orc.draw_distinct(5, 0, n, 3)
    assert got.tolist() == accepted[:3]


def test_signs_balanced(orc):
    s = np.array([orc.sign(2011, c) for c in range(20000)])
    assert set(np.unique(s).tolist()) == {-1.0, 1.0}
    assert abs(s.mean()) < 4.0 / np.sqrt(20000)
