"""The algorithmic byte model behind the bench line's roofline: bytes per
retired transition (8 B fetch of opcode and operand, plus the data word an
ADD or SUB/MUL reads, the word a STORE writes, a READ's tape word and
memory write, and the data word an appending PRINT reads and the output word
it writes; a PRINT past the output capacity moves no word) and the bytes of
building c0, pinned by hand counts."""
import numpy as np
import pytest

import bench
import oracle
from paper_2604_12902_amd import workloads as W


@pytest.mark.parametrize("op,extra", [(1, 0), (2, 4), (3, 4), (4, 4), (5, 0), (6, 8), (7, 0), (8, 0)])
def test_bytes_per_step_of_each_opcode(op, extra):
    mix = np.zeros(16, np.uint64)
    mix[op] = 5
    assert bench.bytes_per_step(mix) == 8.0 + extra


def test_an_appended_print_adds_its_data_and_output_words():
    mix = np.zeros(16, np.uint64)
    mix[7] = 4                      # four PRINTs, one of which appended a word
    mix[9] = 1
    assert bench.bytes_per_step(mix) == pytest.approx(8.0 + 8.0 / 4)


def test_no_retired_step_has_no_bytes():
    assert bench.bytes_per_step(np.zeros(16, np.uint64)) == 0.0


def test_oracle_mix_of_a_hand_traced_program():
    """READ 20; READ 21; LOAD 0; ADD 20; ADD 21; STORE 22; PRINT 22; HALT on
    x = (5, -7) retires two READs, a LOAD, two ADDs, a STORE and one PRINT
    that appends: (7 x 8 + 2 x 8 + 2 x 4 + 4 + 4 + 4) / 7 bytes a step."""
    prog = [6, 20, 6, 21, 1, 0, 2, 20, 2, 21, 4, 22, 7, 22, 0, 0]
    b = W.from_programs(W.ISA_CLASSIC, [prog], 32, [[5, -7]], ell=2, s=4)
    mix = oracle.advance_mix(oracle.init(b), 100)
    assert mix[1:10].tolist() == [1, 2, 0, 1, 0, 2, 1, 0, 1]
    assert bench.bytes_per_step(mix) == pytest.approx(92 / 7)


def test_pack_bytes_by_hand():
    """Two machines, programs of 4 and 6 words, tapes of 2 and 0 words, n = 16,
    l = 3, s = 2: reads 4 (10 + 2) B, writes 4 (2 x 16 + 2 x 3 + 2 x 2) B
    of words and 25 B of scalars per machine."""
    b = W.from_programs(W.ISA_CLASSIC, [[1, 2, 3, 4], [1, 2, 3, 4, 5, 6]], 16, [[7, 8], []],
                        ell=3, s=2)
    assert bench.pack_bytes(b) == 4 * 12 + 4 * 42 + 25 * 2
