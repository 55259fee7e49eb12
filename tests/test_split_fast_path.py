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
