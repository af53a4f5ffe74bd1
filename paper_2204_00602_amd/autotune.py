"""Launch-shape autotuner for single plans and batches.

Times candidate `slos_options_t` settings through the C ABI on the current
device and keeps the fastest.  The search is coordinate descent: starting from
the library defaults, each knob is swept over its candidate values with the
others fixed, the best value is kept, and the sweep repeats until a pass
changes nothing (at most `passes` passes).  Results are cached in a JSON file
keyed by the device name and the workload signature, so a later process picks
the tuned options without timing anything.

    python -m paper_2204_00602_amd.autotune --m 24 --n 12 --dtype c64 --compensated
    python -m paper_2204_00602_amd.autotune --batch 4096 --seed 4
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import inputs, slos

PLAN_SPACE: Dict[str, List[int]] = {
    "leaf_max": [2048, 4096, 8192, 16384, 32768],
    "low_block_max": [2048, 3072, 3584, 4096, 5120],
    "outputs_per_lane": [1, 2, 4],
    "block_threads": [64, 128, 256],
    "grid_blocks": [1024, 2048, 4096, 8192],
    "ticket_leaves": [1, 2, 4],
    "xcd_chunk": [128, 512, 2048],
}

BATCH_SPACE: Dict[str, List[int]] = {
    "leaf_max": [64, 128, 256, 512, 1024, 2048, 4096, 5120, 6144, 8192],
    "outputs_per_lane": [1, 2, 4],
    "block_threads": [64, 128, 256, 512, 1024],
    "grid_blocks": [256, 512, 1024, 2048, 4096],
    "low_block_max": [0, 1536, 2048],
}

# the library defaults the search starts from (0 = library default)
PLAN_START = {"leaf_max": 0, "low_block_max": 0, "outputs_per_lane": 0, "block_threads": 0, "grid_blocks": 0,
              "ticket_leaves": 0, "xcd_chunk": 0}
BATCH_START = {"leaf_max": 0, "outputs_per_lane": 0, "block_threads": 0, "grid_blocks": 0, "low_block_max": 0}


# The tuner's results on MI355X for the benchmark workloads, shipped with the
# package and written by `python -m paper_2204_00602_amd.autotune ... --cache`
# on that device.  tune_plan / tune_batch return an entry found here before
# consulting the per-user cache, so the benchmark times, and the tests check,
# exactly the options recorded here.
SHIPPED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def shipped_options(key: str) -> Optional[dict]:
    """Options shipped for a workload key (see plan_key / batch_key), or None."""
    hit = _load(SHIPPED_PATH).get(key)
    return dict(hit["options"]) if hit else None


def default_cache_path() -> str:
    return os.environ.get("SLOS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "slos_tune.json"))


def _device_name() -> str:
    """The device part of a cache key: architecture and compute-unit count
    (e.g. gfx950-256cu), which do not depend on how the runtime names the
    board (the marketing name differs between processes on one machine)."""
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "") or torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{arch.split(':')[0]}-{props.multi_processor_count}cu"


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: dict):
    data = _load(path)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_ms(run: Callable[[object], None], reps: int, warmup: int) -> float:
    """Median wall time of `run(stream)` between HIP events on one stream."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        run(stream)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run(stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def coordinate_descent(measure: Callable[[dict], Optional[float]], space: Dict[str, List[int]],
                       start: dict, passes: int = 2, log=None) -> tuple:
    """Minimise `measure(options)` one knob at a time.  `measure` returns None
    for a setting the library rejects.  Returns (best options, best ms, trials)."""
    best = dict(start)
    best_ms = measure(best)
    if best_ms is None:
        raise RuntimeError(f"the starting options {best} are rejected")
    seen = {json.dumps(best, sort_keys=True): best_ms}
    for _ in range(passes):
        changed = False
        for knob, values in space.items():
            for v in values:
                cand = dict(best)
                cand[knob] = v
                key = json.dumps(cand, sort_keys=True)
                if key not in seen:
                    seen[key] = measure(cand)
                    if log:
                        log(f"  {cand} -> {seen[key]}")
                ms = seen[key]
                if ms is not None and ms < best_ms:
                    best, best_ms, changed = cand, ms, True
        if not changed:
            break
    return best, best_ms, len(seen)


def plan_key(input_state, dtype: str, compensated: bool) -> str:
    s = np.asarray(input_state, dtype=np.int32)
    return f"plan|{_device_name()}|m={s.size}|T={','.join(map(str, s))}|{dtype}|comp={int(compensated)}"


def batch_key(input_states, dtype: str) -> str:
    h = hashlib.sha256()
    for s in input_states:
        h.update(np.asarray(s, dtype=np.int32).tobytes() + b"|")
    return f"batch|{_device_name()}|count={len(input_states)}|{h.hexdigest()[:16]}|{dtype}"


def tune_plan(input_state: Sequence[int], dtype: str = "c64", compensated: bool = False,
              U=None, reps: int = 3, warmup: int = 1, passes: int = 2, space=None,
              cache: Optional[str] = None, retune: bool = False, log=None) -> dict:
    """Fastest options for `slos.Plan(input_state, dtype, compensated)` on this device."""
    import torch
    cache = cache or default_cache_path()
    key = plan_key(input_state, dtype, compensated)
    if not retune:
        hit = shipped_options(key)
        if hit:
            return hit
        hit = _load(cache).get(key)
        if hit:
            return hit["options"]
    m = len(input_state)
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    Ud = torch.as_tensor(inputs.haar_unitary(m, 0) if U is None else U).to(cdt).cuda().contiguous()
    out = None

    def measure(opts):
        nonlocal out
        try:
            plan = slos.Plan(input_state, dtype, compensated=compensated, options=opts)
        except slos.SlosError:
            return None
        if out is None or out.numel() != plan.num_outputs:
            out = torch.empty(plan.num_outputs, dtype=cdt, device="cuda")
        try:
            return _time_ms(lambda st: plan.amplitudes(Ud, out=out, stream=st), reps, warmup)
        finally:
            plan.close()

    t0 = time.perf_counter()
    best, best_ms, trials = coordinate_descent(measure, space or PLAN_SPACE, PLAN_START, passes, log)
    _store(cache, key, {"options": best, "ms": best_ms, "trials": trials,
                        "seconds": time.perf_counter() - t0})
    return best


def tune_batch(input_states, dtype: str = "c64", Us=None, reps: int = 5, warmup: int = 2,
               passes: int = 2, space=None, cache: Optional[str] = None, retune: bool = False,
               log=None) -> dict:
    """Fastest options for `slos.Batch(input_states, dtype)` on this device."""
    cache = cache or default_cache_path()
    key = batch_key(input_states, dtype)
    if not retune:
        hit = shipped_options(key)
        if hit:
            return hit
        hit = _load(cache).get(key)
        if hit:
            return hit["options"]
    if Us is None:
        Us = [inputs.haar_unitary(len(s), i) for i, s in enumerate(input_states)]
    U = None

    def measure(opts):
        nonlocal U
        try:
            b = slos.Batch(input_states, dtype, options=opts)
        except slos.SlosError:
            return None
        if U is None:
            U = b.pack_u(Us)
        import torch
        out = torch.empty(b.total_outputs, dtype=b._cdt(), device="cuda")
        try:
            return _time_ms(lambda st: b.amplitudes(U, out=out, stream=st), reps, warmup)
        finally:
            b.close()

    t0 = time.perf_counter()
    best, best_ms, trials = coordinate_descent(measure, space or BATCH_SPACE, BATCH_START, passes, log)
    _store(cache, key, {"options": best, "ms": best_ms, "trials": trials,
                        "seconds": time.perf_counter() - t0})
    return best


def main(argv=None):
    ap = argparse.ArgumentParser(description="tune SLOS launch options on this device")
    ap.add_argument("--m", type=int, default=24)
    ap.add_argument("--n", type=int, default=12)
    ap.add_argument("--dtype", choices=["c64", "c128"], default="c64")
    ap.add_argument("--compensated", action="store_true")
    ap.add_argument("--batch", type=int, default=0, help="tune a batch of this many instances instead")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--cache", default=None)
    ap.add_argument("--passes", type=int, default=2)
    args = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    if args.batch:
        inst = inputs.batch_instances(args.batch, seed=args.seed)
        best = tune_batch([t for (_, _, t, _) in inst], args.dtype, Us=[u for (_, _, _, u) in inst],
                          passes=args.passes, cache=args.cache, retune=True, log=log)
        key = batch_key([t for (_, _, t, _) in inst], args.dtype)
    else:
        T = inputs.first_modes_input(args.m, args.n)
        best = tune_plan(T, args.dtype, args.compensated, passes=args.passes, cache=args.cache,
                         retune=True, log=log)
        key = plan_key(T, args.dtype, args.compensated)
    entry = _load(args.cache or default_cache_path())[key]
    print(json.dumps({"key": key, **entry}), flush=True)
    return best


if __name__ == "__main__":
    main()
