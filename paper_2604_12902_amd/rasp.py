"""Python binding of librasp (ctypes).  Argument marshalling only.

Every function here has the name of the C entry point it calls
(``rasp_create``, ``rasp_load_batch``, ``rasp_run``, ``rasp_fetch_outputs``,
...) and does nothing but convert Python objects into the C arguments: all the
work happens in the HIP library.  PyTorch supplies device memory (the arena
and device-resident descriptors) and the stream.  If the built library is
missing, importing this module raises: there is no fallback.

``Context`` bundles the calls for convenience; it adds no behaviour.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
# torch first: it loads the HIP runtime it was built with, and librasp's
# libamdhip64.so.7 then resolves to that same copy, so that device memory and
# streams from torch and the library's calls share one runtime
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librasp.so")

RASP_ABI_VERSION = 4
RASP_OK, RASP_E_INVAL, RASP_E_NOMEM, RASP_E_DEVICE, RASP_E_STATE, RASP_E_BUSY = 0, -1, -2, -3, -4, -5
RASP_ISA_WORD, RASP_ISA_CLASSIC = 0, 1
RASP_RUNNING, RASP_HALTED = 0, 1
RASP_DESC_DEVICE_PTRS = 1
RASP_DESC_LAZY = 2
RASP_OUT_DEVICE_PTRS = 1
RASP_OUT_ASYNC = 2
RASP_OPT_SCHEDULE, RASP_OPT_EPOCH, RASP_OPT_LDS_WORDS = 1, 2, 3
RASP_OPT_WAVES_PER_CU, RASP_OPT_GRAPH, RASP_OPT_FIRST_PASS = 4, 5, 6
RASP_SCHED_AUTO, RASP_SCHED_PLAIN, RASP_SCHED_PERSISTENT = 0, 1, 2
RASP_OPT_PROFILE = 7
RASP_OPT_FIRST_PASS_KIND = 8
RASP_OPT_HOT_CELLS = 9
RASP_OPT_PROFILE_STEPS = 10
RASP_OPT_MISFIT_WAVES = 11
KERNEL_NAMES = ("pack", "plain", "persistent", "digest", "other", "first", "misfit")

EXPORTED = ("rasp_create", "rasp_create_on_cus", "rasp_destroy", "rasp_last_error", "rasp_batch_footprint",
            "rasp_load_batch", "rasp_load_state", "rasp_run", "rasp_run_multi", "rasp_run_async",
            "rasp_run_noalloc",
            "rasp_poll", "rasp_sync", "rasp_fetch_outputs", "rasp_batch_info",
            "rasp_free_batch", "rasp_set_option", "rasp_get_option", "rasp_device_info",
            "rasp_kernel_times", "rasp_running_counts", "rasp_running_counts_async",
            "rasp_running_counts_wait", "rasp_autotune")

_ERRNAMES = {RASP_E_INVAL: "RASP_E_INVAL", RASP_E_NOMEM: "RASP_E_NOMEM",
             RASP_E_DEVICE: "RASP_E_DEVICE", RASP_E_STATE: "RASP_E_STATE",
             RASP_E_BUSY: "RASP_E_BUSY"}

P = ctypes.c_void_p


class rasp_batch_desc(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("isa", ctypes.c_uint32),
                ("num_vms", ctypes.c_uint64),
                ("prog", P), ("prog_off", P), ("mem_words", P),
                ("default_mem_words", ctypes.c_uint32), ("default_out_cap", ctypes.c_uint32),
                ("tape", P), ("tape_off", P), ("tape_cap", P), ("out_cap", P),
                ("flags", ctypes.c_uint32), ("word_bits", ctypes.c_uint32)]


class rasp_outputs(ctypes.Structure):
    _fields_ = [("status", P), ("steps", P), ("i", P), ("a", P), ("u0", P), ("y0", P),
                ("y", P), ("mem", P), ("mem_digest", P),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class RaspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_ERRNAMES.get(code, str(code)), msg))
        self.code = code


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("librasp.so is not built (run paper_2604_12902_amd.build.build())")
    lib = ctypes.CDLL(path)
    u64, i64, u32, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int
    sig = {
        "rasp_create": ([ctypes.POINTER(P), i32, P, u64, P], i32),
        "rasp_create_on_cus": ([ctypes.POINTER(P), i32, P, u64, u32, u32], i32),
        "rasp_destroy": ([P], i32),
        "rasp_last_error": ([P], ctypes.c_char_p),
        "rasp_batch_footprint": ([ctypes.POINTER(rasp_batch_desc), ctypes.POINTER(u64)], i32),
        "rasp_load_batch": ([P, ctypes.POINTER(rasp_batch_desc), ctypes.POINTER(u64)], i32),
        "rasp_load_state": ([P, ctypes.POINTER(rasp_batch_desc), ctypes.POINTER(rasp_outputs),
                             ctypes.POINTER(u64)], i32),
        "rasp_run": ([P, u64, u64], i32),
        "rasp_run_multi": ([P, P, P, u32], i32),
        "rasp_run_async": ([P, P, P, u32], i32),
        "rasp_run_noalloc": ([P, u64, u64], i32),
        "rasp_poll": ([P, u64, ctypes.POINTER(i32)], i32),
        "rasp_sync": ([P, u64], i32),
        "rasp_fetch_outputs": ([P, u64, ctypes.POINTER(rasp_outputs)], i32),
        "rasp_batch_info": ([P, u64, P, P, P, P], i32),
        "rasp_free_batch": ([P, u64], i32),
        "rasp_set_option": ([P, i32, i64], i32),
        "rasp_get_option": ([P, i32, ctypes.POINTER(i64)], i32),
        "rasp_device_info": ([P, P, P, P], i32),
        "rasp_kernel_times": ([P, P, P], i32),
        "rasp_running_counts": ([P, P, u32, P], i32),
        "rasp_running_counts_async": ([P, P, u32, ctypes.POINTER(u64)], i32),
        "rasp_running_counts_wait": ([P, u64, P], i32),
        "rasp_autotune": ([P, u64, u64, u64, P, P], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = load_library()


def _check(rc, ctx=None):
    if rc != RASP_OK:
        msg = _lib.rasp_last_error(ctx)
        raise RaspError(rc, msg.decode() if msg else "")
    return rc


def _ptr(x):
    """Address of a numpy array or a torch tensor (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


# ---- descriptors ------------------------------------------------------------------

@dataclass
class Desc:
    """A rasp_batch_desc plus the arrays it points at (kept alive)."""
    c: rasp_batch_desc
    keep: tuple


def make_desc(batch, device=None, lazy: bool = False) -> Desc:
    """Descriptor for a workloads.Batch.  With device=<torch device> the arrays are
    copied to the GPU first and the descriptor says RASP_DESC_DEVICE_PTRS (plus
    RASP_DESC_LAZY when lazy: c0 is then built by the first run)."""
    arrs = dict(prog=np.ascontiguousarray(batch.prog, np.int32),
                prog_off=np.ascontiguousarray(batch.prog_off, np.uint64),
                mem_words=np.ascontiguousarray(batch.mem_words, np.uint32),
                tape=np.ascontiguousarray(batch.tape, np.int32),
                tape_off=np.ascontiguousarray(batch.tape_off, np.uint64),
                tape_cap=np.ascontiguousarray(batch.tape_cap, np.uint32),
                out_cap=np.ascontiguousarray(batch.out_cap, np.uint32))
    flags = 0
    if device is not None:
        import torch
        signed = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32}
        arrs = {k: torch.from_numpy(v.view(signed.get(v.dtype, v.dtype))).to(device)
                for k, v in arrs.items()}
        flags = RASP_DESC_DEVICE_PTRS | (RASP_DESC_LAZY if lazy else 0)
    return desc_from_arrays(batch.isa, batch.N, flags=flags,
                            word_bits=getattr(batch, "word_bits", 32), **arrs)


def desc_from_arrays(isa, num_vms, prog, prog_off, tape, tape_off, mem_words=None,
                     default_mem_words=0, tape_cap=None, out_cap=None, default_out_cap=0,
                     flags=0, word_bits=32) -> Desc:
    c = rasp_batch_desc(RASP_ABI_VERSION, isa, num_vms, _ptr(prog), _ptr(prog_off),
                        _ptr(mem_words), default_mem_words, default_out_cap, _ptr(tape),
                        _ptr(tape_off), _ptr(tape_cap), _ptr(out_cap), flags, word_bits)
    return Desc(c, (prog, prog_off, mem_words, tape, tape_off, tape_cap, out_cap))


# ---- the C entry points ------------------------------------------------------------

def rasp_create(device: int, arena, arena_bytes: int, stream) -> int:
    """arena: a torch uint8 CUDA tensor (or None: library allocates); stream: a
    torch.cuda.Stream, an int handle, or None."""
    out = P()
    sh = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    rc = _lib.rasp_create(ctypes.byref(out), device, _ptr(arena), arena_bytes, sh)
    _check(rc)
    return out.value


def rasp_create_on_cus(device: int, arena, arena_bytes: int, cu_first: int, cu_count: int) -> int:
    """A context on its own stream restricted to compute units
    [cu_first, cu_first + cu_count)."""
    out = P()
    _check(_lib.rasp_create_on_cus(ctypes.byref(out), device, _ptr(arena), arena_bytes, cu_first, cu_count))
    return out.value


def rasp_destroy(ctx) -> None:
    _check(_lib.rasp_destroy(ctx))


def rasp_last_error(ctx) -> str:
    m = _lib.rasp_last_error(ctx)
    return m.decode() if m else ""


def rasp_batch_footprint(desc: Desc) -> int:
    out = ctypes.c_uint64()
    _check(_lib.rasp_batch_footprint(ctypes.byref(desc.c), ctypes.byref(out)))
    return out.value


def rasp_load_batch(ctx, desc: Desc) -> int:
    h = ctypes.c_uint64()
    _check(_lib.rasp_load_batch(ctx, ctypes.byref(desc.c), ctypes.byref(h)), ctx)
    return h.value


def _outputs_struct(d: dict, flags=0) -> rasp_outputs:
    return rasp_outputs(*[_ptr(d.get(k)) for k in
                          ("status", "steps", "i", "a", "u0", "y0", "y", "mem", "mem_digest")],
                        flags, 0)


def rasp_load_state(ctx, desc: Desc, state: dict) -> int:
    """state: dict of numpy arrays i, a, u0, y0, mem (required), steps, y."""
    st = {k: np.ascontiguousarray(v) for k, v in state.items()}
    s = _outputs_struct(st)
    h = ctypes.c_uint64()
    _check(_lib.rasp_load_state(ctx, ctypes.byref(desc.c), ctypes.byref(s), ctypes.byref(h)), ctx)
    return h.value


def rasp_run(ctx, batch: int, budget: int) -> None:
    _check(_lib.rasp_run(ctx, batch, budget), ctx)


def rasp_run_noalloc(ctx, batch: int, budget: int) -> None:
    _check(_lib.rasp_run_noalloc(ctx, batch, budget), ctx)


def rasp_run_multi(ctx, batches, budgets) -> None:
    hs = np.ascontiguousarray(batches, np.uint64)
    bs = np.ascontiguousarray(budgets, np.uint64)
    _check(_lib.rasp_run_multi(ctx, _ptr(hs), _ptr(bs), len(hs)), ctx)


def rasp_run_async(ctx, batches, budgets) -> None:
    hs = np.ascontiguousarray(batches, np.uint64)
    bs = np.ascontiguousarray(budgets, np.uint64)
    _check(_lib.rasp_run_async(ctx, _ptr(hs), _ptr(bs), len(hs)), ctx)


def rasp_poll(ctx, batch: int = 0) -> bool:
    done = ctypes.c_int()
    _check(_lib.rasp_poll(ctx, batch, ctypes.byref(done)), ctx)
    return bool(done.value)


def rasp_sync(ctx, batch: int = 0) -> None:
    _check(_lib.rasp_sync(ctx, batch), ctx)


def rasp_batch_info(ctx, batch: int, steps_sum: bool = False) -> dict:
    vals = [ctypes.c_uint64() for _ in range(4)]
    _check(_lib.rasp_batch_info(ctx, batch, ctypes.byref(vals[0]), ctypes.byref(vals[1]),
                                ctypes.byref(vals[2]),
                                ctypes.byref(vals[3]) if steps_sum else None), ctx)
    out = dict(num_vms=vals[0].value, mem_words=vals[1].value, out_words=vals[2].value)
    if steps_sum:
        out["steps_sum"] = vals[3].value
    return out


def rasp_fetch_outputs(ctx, batch: int, mem: bool = False, digest: bool = False,
                       fields=("status", "steps", "i", "a", "u0", "y0", "y")) -> dict:
    """Fetch into freshly allocated numpy arrays."""
    info = rasp_batch_info(ctx, batch)
    N = info["num_vms"]
    dt = dict(status=np.uint8, steps=np.uint64, i=np.int32, a=np.int32, u0=np.uint32,
              y0=np.uint32)
    out = {k: np.zeros(N, dt[k]) for k in fields if k in dt}
    if "y" in fields:
        out["y"] = np.zeros(info["out_words"], np.int32)
    if mem:
        out["mem"] = np.zeros(info["mem_words"], np.int32)
    if digest:
        out["mem_digest"] = np.zeros(N, np.uint64)
    s = _outputs_struct(out)
    _check(_lib.rasp_fetch_outputs(ctx, batch, ctypes.byref(s)), ctx)
    return out


def rasp_fetch_outputs_into(ctx, batch: int, dst: dict, device: bool) -> None:
    """Fetch into caller-owned buffers (numpy or torch device tensors)."""
    s = _outputs_struct(dst, RASP_OUT_DEVICE_PTRS if device else 0)
    _check(_lib.rasp_fetch_outputs(ctx, batch, ctypes.byref(s)), ctx)


def rasp_running_counts(ctx, batches) -> np.ndarray:
    hs = np.ascontiguousarray(batches, np.uint64)
    out = np.zeros(len(hs), np.uint64)
    _check(_lib.rasp_running_counts(ctx, _ptr(hs), len(hs), _ptr(out)), ctx)
    return out


def rasp_running_counts_async(ctx, batches) -> tuple:
    """Queue the running counts of `batches`; returns (ticket, number of batches)."""
    hs = np.ascontiguousarray(batches, np.uint64)
    t = ctypes.c_uint64()
    _check(_lib.rasp_running_counts_async(ctx, _ptr(hs), len(hs), ctypes.byref(t)), ctx)
    return t.value, len(hs)


def rasp_running_counts_wait(ctx, ticket: tuple) -> np.ndarray:
    out = np.zeros(ticket[1], np.uint64)
    _check(_lib.rasp_running_counts_wait(ctx, ticket[0], _ptr(out)), ctx)
    return out


def pinned_outputs(info: dict, digest: bool = True,
                   fields=("status", "steps", "i", "a", "u0", "y0", "y")) -> dict:
    """Page-locked host buffers (torch pinned tensors) for an asynchronous
    fetch of a batch with rasp_batch_info `info`; numpy views of them stay
    valid while the dict is alive."""
    import torch
    N = info["num_vms"]
    dt = dict(status=torch.uint8, steps=torch.int64, i=torch.int32, a=torch.int32, u0=torch.int32,
              y0=torch.int32)
    out = {k: torch.empty(N, dtype=dt[k], pin_memory=True) for k in fields if k in dt}
    if "y" in fields:
        out["y"] = torch.empty(max(1, info["out_words"]), dtype=torch.int32, pin_memory=True)
    if digest:
        out["mem_digest"] = torch.empty(N, dtype=torch.int64, pin_memory=True)
    return out


def rasp_fetch_outputs_async(ctx, batch: int, dst: dict) -> None:
    """Queue a fetch into page-locked host buffers (pinned_outputs); the
    buffers are filled when rasp_poll(ctx, batch) reports the batch done."""
    s = _outputs_struct(dst, RASP_OUT_ASYNC)
    _check(_lib.rasp_fetch_outputs(ctx, batch, ctypes.byref(s)), ctx)


def outputs_as_numpy(dst: dict, info: dict) -> dict:
    """numpy copies of a completed asynchronous fetch, with the dtypes of
    rasp_fetch_outputs."""
    dt = dict(status=np.uint8, steps=np.uint64, i=np.int32, a=np.int32, u0=np.uint32, y0=np.uint32,
              y=np.int32, mem_digest=np.uint64)
    out = {k: v.numpy().view(dt[k]).copy() for k, v in dst.items()}
    if "y" in out:
        out["y"] = out["y"][:info["out_words"]]
    return out


AUTOTUNE_KNOBS = ("schedule", "lds_words", "first_pass", "epoch", "waves_per_cu",
                  "first_pass_kind", "hot_cells", "profile_steps", "misfit_waves")


def rasp_autotune(ctx, batch: int, budget: int, max_vms: int = 0) -> dict:
    """Pick and set the scheduling knobs for batches shaped like `batch`."""
    chosen = np.zeros(len(AUTOTUNE_KNOBS), np.int64)
    best = ctypes.c_double()
    _check(_lib.rasp_autotune(ctx, batch, budget, max_vms, _ptr(chosen), ctypes.byref(best)), ctx)
    out = {k: int(v) for k, v in zip(AUTOTUNE_KNOBS, chosen)}
    out["best_ms"] = best.value
    return out


def rasp_free_batch(ctx, batch: int) -> None:
    _check(_lib.rasp_free_batch(ctx, batch), ctx)


def rasp_set_option(ctx, option: int, value: int) -> None:
    _check(_lib.rasp_set_option(ctx, option, value), ctx)


def rasp_get_option(ctx, option: int) -> int:
    v = ctypes.c_int64()
    _check(_lib.rasp_get_option(ctx, option, ctypes.byref(v)), ctx)
    return v.value


def rasp_device_info(ctx) -> dict:
    cu, lds, wv = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lib.rasp_device_info(ctx, ctypes.byref(cu), ctypes.byref(lds), ctypes.byref(wv)), ctx)
    return dict(compute_units=cu.value, lds_bytes=lds.value, wave_size=wv.value)


def rasp_kernel_times(ctx) -> dict:
    """{kernel kind: (total ms, launches)} recorded since the last call."""
    ms = np.zeros(len(KERNEL_NAMES), np.float64)
    n = np.zeros(len(KERNEL_NAMES), np.uint64)
    _check(_lib.rasp_kernel_times(ctx, _ptr(ms), _ptr(n)), ctx)
    return {k: (float(ms[j]), int(n[j])) for j, k in enumerate(KERNEL_NAMES)}


# ---- convenience wrapper -------------------------------------------------------------

class Context:
    """Owns a torch-allocated arena and a context on one device."""

    def __init__(self, arena_bytes: int, device: int = 0, stream=None, cus=None):
        """cus = (first, count): the context's own stream runs on those compute
        units only (rasp_create_on_cus); otherwise on `stream`, or a new torch
        stream."""
        import torch
        self.device = torch.device("cuda", device)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=self.device)
        if cus is not None:
            self.stream = None
            self.handle = rasp_create_on_cus(device, self.arena, arena_bytes, int(cus[0]), int(cus[1]))
        else:
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.handle = rasp_create(device, self.arena, arena_bytes, self.stream)
        self._keep = {}

    def close(self):
        if self.handle:
            rasp_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, batch, device_desc: bool = False, lazy: bool = False) -> int:
        """Load a batch.  A lazy descriptor (device arrays read by the first
        run) is kept alive here until the batch is freed."""
        d = make_desc(batch, self.device if (device_desc or lazy) else None, lazy=lazy)
        h = rasp_load_batch(self.handle, d)
        if lazy:
            self._keep[h] = d
        return h

    def load_state(self, batch, state: dict) -> int:
        return rasp_load_state(self.handle, make_desc(batch), state)

    def run(self, b: int, budget: int) -> None:
        rasp_run(self.handle, b, budget)

    def run_multi(self, bs, budgets) -> None:
        rasp_run_multi(self.handle, bs, budgets)

    def fetch(self, b: int, mem: bool = False, digest: bool = False) -> dict:
        return rasp_fetch_outputs(self.handle, b, mem=mem, digest=digest)

    def free(self, b: int) -> None:
        rasp_free_batch(self.handle, b)
        self._keep.pop(b, None)

    def sync(self, b: int = 0) -> None:
        rasp_sync(self.handle, b)

    def poll(self, b: int = 0) -> bool:
        return rasp_poll(self.handle, b)

    def info(self, b: int, steps_sum: bool = False) -> dict:
        return rasp_batch_info(self.handle, b, steps_sum)

    def set(self, option: int, value: int) -> None:
        rasp_set_option(self.handle, option, value)

    def get(self, option: int) -> int:
        return rasp_get_option(self.handle, option)


def cu_share(k: int, n: int, cus: int):
    """(first, count) of the k-th of n contiguous shares of `cus` compute units."""
    first = -(-k * cus // n)
    return first, -(-(k + 1) * cus // n) - first
