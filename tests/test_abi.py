"""The C ABI library loads and exports every entry point its header declares
(no compute call: these run without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rasp.h")
LIB = os.path.join(ROOT, "paper_2604_12902_amd", "librasp.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rasp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("rasp_load_batch", "rasp_run", "rasp_fetch_outputs", "rasp_create",
                 "rasp_destroy", "rasp_run_multi", "rasp_load_state"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_uses_the_c_names():
    from paper_2604_12902_amd import rasp
    for n in declared():
        assert n in rasp.EXPORTED, n
        assert callable(getattr(rasp, n)), n


def test_last_error_without_context_is_callable():
    lib = ctypes.CDLL(LIB)
    lib.rasp_last_error.restype = ctypes.c_char_p
    lib.rasp_last_error.argtypes = [ctypes.c_void_p]
    assert isinstance(lib.rasp_last_error(None), bytes)


def test_footprint_is_pure_and_checks_descriptors():
    """rasp_batch_footprint touches no device for a host descriptor."""
    import numpy as np
    from paper_2604_12902_amd import rasp, workloads as W
    b = W.config1(num_vms=10)
    fp = rasp.rasp_batch_footprint(rasp.make_desc(b))
    words = int(b.mem_words.sum() + b.tape_cap.sum() + b.out_cap.sum())
    assert fp >= 4 * words + 25 * 10
    bad = W.config1(num_vms=10)
    bad.mem_words = np.full(10, 4, np.uint32)            # program longer than memory
    try:
        rasp.rasp_batch_footprint(rasp.make_desc(bad))
        raise AssertionError("expected RASP_E_INVAL")
    except rasp.RaspError as e:
        assert e.code == rasp.RASP_E_INVAL


def test_binding_constants_match_the_header():
    """Every RASP_* constant of the header has the same value in the binding."""
    from paper_2604_12902_amd import rasp
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    consts = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(RASP_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)}
    m = re.search(r"#define\s+RASP_ABI_VERSION\s+(\d+)u", src)
    consts["RASP_ABI_VERSION"] = int(m.group(1))
    assert len(consts) > 30
    for name, value in consts.items():
        if name.startswith("RASP_KERNEL_"):
            continue
        assert getattr(rasp, name) == value, name
    kinds = {n: v for n, v in consts.items() if n.startswith("RASP_KERNEL_") and n != "RASP_KERNEL_COUNT"}
    assert consts["RASP_KERNEL_COUNT"] == len(rasp.KERNEL_NAMES) == len(kinds)
    for n, v in kinds.items():
        assert rasp.KERNEL_NAMES[v] == n[len("RASP_KERNEL_"):].lower(), n


def test_cu_shares_tile_the_device():
    from paper_2604_12902_amd import rasp
    for cus in (256, 255, 80, 7):
        for n in (1, 2, 3, 4):
            shares = [rasp.cu_share(k, n, cus) for k in range(n)]
            assert shares[0][0] == 0
            for (f0, c0), (f1, _) in zip(shares, shares[1:]):
                assert f0 + c0 == f1
            assert sum(c for _, c in shares) == cus
            assert max(c for _, c in shares) - min(c for _, c in shares) <= 1
