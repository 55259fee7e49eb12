"""The seeded workload generators: determinism and the stated distributions."""
import numpy as np

from paper_2604_12902_amd import dsl, workloads as W


def test_same_seed_same_bytes():
    assert W.config1().sha256() == W.config1().sha256()
    assert W.config1(seed=1).sha256() != W.config1().sha256()
    assert W.config3(num_vms=500).sha256() == W.config3(num_vms=500).sha256()


def test_plain_small_shape_and_ranges():
    b = W.config1()
    assert b.N == 4096 and b.budget == 256
    prog = b.prog.reshape(b.N, 32)
    assert prog[:, 0::2].min() == 0 and prog[:, 0::2].max() == 8
    assert prog[:, 1::2].min() == 0 and prog[:, 1::2].max() == 31
    assert b.tape.min() == -8 and b.tape.max() == 8
    assert (b.mem_words == 32).all() and (b.tape_cap == 8).all() and (b.out_cap == 256).all()
    counts = np.bincount(prog[:, 0::2].ravel(), minlength=9)
    assert counts.min() > 0.9 * counts.mean()


def test_plain_scale_shape():
    b = W.config2(num_vms=1000)
    assert b.prog.size == 1000 * 128 and b.budget == 4096
    assert b.prog[1::2].max() == 255 and (b.mem_words == 256).all()
    assert b.tape.min() == -100 and b.tape.max() == 100


def test_uneven_batch_structure():
    b = W.config3(num_vms=3000)
    L = (np.diff(b.prog_off.astype(np.int64)) // 2)
    assert L.min() >= 8 and L.max() <= 512
    assert (b.mem_words >= 2 * L).all() and b.mem_words.max() <= 1024 and b.mem_words.min() >= 64
    back = fwd = 0
    for v in range(b.N):
        p = b.prog[int(b.prog_off[v]):int(b.prog_off[v + 1])]
        ops, opd = p[0::2], p[1::2]
        assert (ops == W.HALT).sum() == 1
        jumps = np.flatnonzero((ops == W.JMP) | (ops == W.JPOS))
        assert (opd[jumps] % 2 == 0).all()
        assert (opd[jumps] <= 2 * L[v]).all()
        back += int((opd[jumps] <= 2 * jumps).sum())
        fwd += int((opd[jumps] > 2 * jumps).sum())
        data = np.flatnonzero((ops != W.JMP) & (ops != W.JPOS) & (ops != W.HALT))
        assert (opd[data] >= 0).all() and (opd[data] < b.mem_words[v]).all()
    assert 0.12 < back / (back + fwd) < 0.18
    # log-uniform lengths: the median is near sqrt(8 * 513)
    assert 45 < np.median(L) < 85


def test_rollout_programs_fit_and_have_stated_lengths():
    b = W.config4(num_vms=40, num_distinct=40)
    L = np.diff(b.prog_off.astype(np.int64)) // 2
    assert L.min() >= 128 and L.max() <= 384
    for d in range(40):
        pairs, data = dsl.lower_classic(W.rollout_program(3, d))
        assert 2 * len(pairs) + data <= W.ROLLOUT_MEM
    assert b.tape.min() >= -(1 << 15) and b.tape.max() < (1 << 15)


def test_subset_roundtrip():
    b = W.config3(num_vms=200)
    idx = np.array([5, 3, 199, 0])
    s = b.subset(idx)
    for k, v in enumerate(idx):
        assert np.array_equal(s.prog[int(s.prog_off[k]):int(s.prog_off[k + 1])],
                              b.prog[int(b.prog_off[v]):int(b.prog_off[v + 1])])


def test_batch_file_round_trip(tmp_path):
    b = W.config3(num_vms=300, budget=777)
    b.meta["workload"] = "uneven"
    path = str(tmp_path / "b.npz")
    W.save_batch(b, path)
    c = W.load_batch(path)
    assert c.sha256() == b.sha256() and c.budget == 777 and c.name == b.name
    assert c.meta["workload"] == "uneven" and c.isa == b.isa and c.word_bits == 32
