"""The split-slot step loop's common case, checked exhaustively on small
memories: whenever a lane's largest position in use -- its data position if
it stores or reads its data word, its next instruction np and np + 1 -- stays
below min(n, P) (and i is not within 4 of the largest word), the positions
the loop computes without division equal the Euclidean ones, and the next
instruction's two words are M[np] and M[(np + 1) mod n] = M[np + 1] inside the
slot.  A model of the loop's position arithmetic, in numpy (32-bit words)."""
import numpy as np


def _emod(v, n):
    return np.mod(v, n)                     # numpy's mod of int64 by n > 0 is Euclidean


def test_fast_path_positions_are_exact():
    js = np.arange(-70, 90, dtype=np.int64)
    for n in range(2, 41):
        for P in range(4, 45, 4):
            lim = min(n, P)
            for pow2 in ((False, True) if n & (n - 1) == 0 else (False,)):
                for p in range(n):
                    i = p + 3 * n                   # any i with i mod n = p, far from the top
                    for taken in (False, True):
                        for uses in (False, True):
                            ju = js & 0xFFFFFFFF        # the word as the loop's uint32
                            if pow2:
                                jj = ju & (n - 1)
                                seq = (p + 2) & (n - 1)
                            else:
                                jj = ju
                                seq = p + 2 - n if p + 2 >= n else p + 2
                            np_ = jj if taken else np.full_like(jj, seq)
                            jx = jj if uses else np.zeros_like(jj)
                            fast = np.maximum(np.maximum(jx, np_), np_ + 1) < lim
                            if not fast.any():
                                continue
                            j = js[fast]
                            if uses:
                                assert (jj[fast] == _emod(j, n)).all() and (jj[fast] < P).all()
                            want_np = _emod(j, n) if taken else np.full(j.shape, _emod(i + 2, n))
                            got_np = np_[fast]
                            assert (got_np == want_np).all(), (n, P, p, taken, pow2)
                            # the two-word read at np: operand position (np + 1) mod n
                            assert (got_np + 1 == _emod(want_np + 1, n)).all()
                            assert (got_np + 1 < P).all()


def test_common_positions_of_the_other_loops_are_exact():
    """Memory in HBM or whole in LDS: a lane is rare when j is outside [0, n),
    i is within 4 of the largest word, or n < 2; otherwise jj = j, the next
    instruction and its operand (wrapping to word 0) are the Euclidean ones."""
    js = np.arange(-70, 90, dtype=np.int64)
    for n in range(2, 41):
        for p in range(n):
            i = p + 5 * n
            for taken in (False, True):
                ju = js & 0xFFFFFFFF
                rare = ju >= n
                seq = p + 2 - n if p + 2 >= n else p + 2
                np_ = np.where(taken, ju, seq)
                nq = np.where(np_ + 1 == n, 0, np_ + 1)
                j = js[~rare]
                assert (ju[~rare] == _emod(j, n)).all()
                want_np = _emod(j, n) if taken else np.full(j.shape, _emod(i + 2, n))
                assert (np_[~rare] == want_np).all()
                assert (nq[~rare] == _emod(want_np + 1, n)).all()


def test_lockstep_euclidean_remainder_is_exact():
    """The lockstep loops reduce an operand outside [0, n) (n not a power of
    two, 2 <= n <= 2^30) without a division: a negative word is moved up by
    big = n * ceil(2^31 / n) into [0, 2^32), then r = u - mulhi(u, rinv) * n
    with rinv = floor((2^32 - 1) / n) is below 2n, and one subtraction of n
    finishes.  A model of that arithmetic in numpy (uint64 for the products)
    against the Euclidean remainder, on the int32 edges and random words."""
    rng = np.random.Generator(np.random.PCG64(7))
    edges = np.array([0, 1, -1, 2, -2, 2 ** 31 - 1, -2 ** 31, 2 ** 31 - 2, -2 ** 31 + 1], np.int64)
    ns = np.concatenate([np.arange(2, 300), rng.integers(2, 2 ** 30 + 1, 300),
                         [3, 641, 1000, 2 ** 30 - 1, 2 ** 30, 2 ** 29 + 3]]).astype(np.int64)
    words = np.concatenate([edges, rng.integers(-2 ** 31, 2 ** 31, 2000)])
    for n in ns:
        rinv = np.uint64((2 ** 32 - 1) // int(n))
        big = np.uint64(((2 ** 31 + int(n) - 1) // int(n)) * int(n))
        assert big < 2 ** 32
        u = (words & 0xFFFFFFFF).astype(np.uint64) + np.where(words < 0, big, np.uint64(0))
        u &= np.uint64(0xFFFFFFFF)
        q = (u * rinv) >> np.uint64(32)
        rr = u - q * np.uint64(n)
        assert (rr < 2 * n).all()
        got = np.where(rr >= np.uint64(n), rr - np.uint64(n), rr)
        assert (got.astype(np.int64) == _emod(words, n)).all(), n
