"""Autotuner of the library's launch choices, cached as JSON by problem shape.

Rows of the adaptive setup are independent (Sec. 2), so the setup of a matrix, or of a batch
of systems concatenated block-diagonally, is one launch whose shape is free: how many lanes
own a row (8, 16 or 64: 8, 4 or 1 rows per wavefront), how many slots the first on-chip
candidate table has, and how many wavefronts' worth of rows one claim takes.  The PCG
iteration (Sec. 5.2) has its own: whether the products also form the updated vectors (fused)
or separate update kernels run, whether each iteration is replayed from a captured HIP graph,
and the SELL-64 layout of G^T's uneven rows (rows ordered by length in windows of four slices,
or split layouts).

Every choice here leaves the results of a form unchanged: any lanes / table / claim give the
setup's G bit for bit, fused or separate kernels and graph replay give the iterates bit for
bit, and the two G^T layouts give the products row by row bit for bit (their fused dot
products are summed in another order, so iterates agree to rounding).  The tuner times each
candidate with the library's own timers (the setup's and the solve's wall time on the
device), keeps the fastest, and caches the choice in a JSON file keyed by the problem shape,
so that later runs of the same shape apply it without measuring.

Options are process-wide (``afsai_set_option``): ``apply(choice)`` sets them for the calls
inside its ``with`` block and restores the automatic choices afterwards.
"""
from __future__ import annotations

import contextlib
import json
import os
import statistics

import numpy as np

from . import (OPT_PCG_FORM, OPT_PCG_GRAPH, OPT_SELL_UNEVEN, OPT_SETUP_CLAIM, OPT_SETUP_LANES, OPT_SETUP_TABLE,
               pcg_solve, pcg_solve_batched, set_option, setup, setup_batched)

SETUP_KEYS = {"lanes": OPT_SETUP_LANES, "table": OPT_SETUP_TABLE, "claim": OPT_SETUP_CLAIM}
PCG_KEYS = {"pcg_form": OPT_PCG_FORM, "pcg_graph": OPT_PCG_GRAPH, "gt_layout": OPT_SELL_UNEVEN}

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2010_14175_amd", "tune.json")


def shape_key(n: int, nnz: int, maxlen: int, nsys: int, kmax: int, s: int, g_prec: int) -> str:
    """The shape a choice is cached under: rows, entries, longest row, systems, pattern
    parameters and storage of G."""
    return f"n{n}_nnz{nnz}_len{maxlen}_sys{nsys}_k{kmax}_s{s}_g{g_prec}"


@contextlib.contextmanager
def apply(choice: dict | None):
    """Sets the options of a tuned choice for the calls inside the block."""
    opts = {}
    for part, keys in (("setup", SETUP_KEYS), ("pcg", PCG_KEYS)):
        for name, val in ((choice or {}).get(part) or {}).items():
            opts[keys[name]] = int(val)
    try:
        for o, v in opts.items():
            set_option(o, v)
        yield
    finally:
        for o in opts:
            set_option(o, 0)


def _lane_choices(mmax: int, maxlen: int) -> list[int]:
    lanes = []
    if mmax <= 8 and maxlen <= 16:
        lanes.append(8)
    if mmax <= 16 and maxlen <= 64:
        lanes.append(16)
    return lanes + [64]


def _median_ms(fn, reps: int) -> float:
    fn()  # warm-up
    return statistics.median(fn() for _ in range(reps))


def autotune(dA, kmax: int, s: int, eps: float, b, g_prec: int = 0, offsets=None, rtol: float = 1e-8,
             reps: int = 2, cache: str | None = DEFAULT_CACHE, verbose: bool = False) -> dict:
    """The fastest setup and PCG choices for this problem (a matrix, or a batch when offsets
    are given), from the cache when its shape is there.  Returns
    {"key", "setup": {...}, "pcg": {...}, "setup_ms", "pcg_ms", "default_setup_ms",
    "default_pcg_ms"}."""
    import torch

    rp = dA.row_ptr.cpu().numpy()
    maxlen = int(np.max(np.diff(rp)))
    nsys = 1 if offsets is None else len(offsets) - 1
    key = shape_key(dA.n, dA.nnz, maxlen, nsys, kmax, s, g_prec)
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            store = json.load(fh)
        if key in store:
            return store[key]
    mmax = 1 + kmax * s

    def do_setup():
        if offsets is None:
            return setup(dA, kmax, s, eps, g_prec=g_prec)
        return setup_batched(dA, offsets, kmax, s, eps, g_prec=g_prec)

    def time_setup():
        P = do_setup()
        ms = P.info().ms
        P.close()
        return ms

    x = torch.zeros_like(b)

    def time_pcg(P):
        x.zero_()
        if offsets is None:
            _, info = pcg_solve(dA, P, b, x=x, rtol=rtol)
            return info.ms
        _, infos = pcg_solve_batched(dA, P, offsets, b, x=x, rtol=rtol)
        return infos[0].ms

    # setup: one knob at a time (lanes per row, then table slots, then rows per claim), each
    # from the best choice so far
    res_setup = []

    def trial(c):
        try:
            with apply({"setup": c}):
                ms = _median_ms(time_setup, reps)
        except Exception:  # a shape the choice does not support
            return None
        res_setup.append((ms, c))
        if verbose:
            print(f"[tune] setup {c}: {ms:.3f} ms")
        return ms

    best_setup, best_setup_ms = {}, trial({})
    for name, values in (("lanes", _lane_choices(mmax, maxlen)), ("table", (128, 256, 512, 1024)),
                         ("claim", (1, 2, 4, 8, 16, 32))):
        for v in values:
            c = dict(best_setup, **{name: v})
            ms = trial(c)
            if ms is not None and ms < best_setup_ms:
                best_setup, best_setup_ms = c, ms
    with apply({"setup": best_setup}):
        P = do_setup()
    res_pcg = []
    for form in (0, 1, 2):
        for graph in (0, 2):
            for layout in (0, 1):
                c = {k: v for k, v in (("pcg_form", form), ("pcg_graph", graph), ("gt_layout", layout)) if v}
                try:
                    with apply({"pcg": c}):
                        if layout:  # the layout of G^T is built by the setup
                            with apply({"setup": best_setup}):
                                Pc = do_setup()
                            ms = _median_ms(lambda: time_pcg(Pc), reps)
                            Pc.close()
                        else:
                            ms = _median_ms(lambda: time_pcg(P), reps)
                except Exception:
                    continue
                res_pcg.append((ms, c))
                if verbose:
                    print(f"[tune] pcg {c}: {ms:.3f} ms")
    P.close()
    best_pcg_ms, best_pcg = min(res_pcg, key=lambda t: t[0])
    choice = {"key": key, "setup": best_setup, "pcg": best_pcg, "setup_ms": round(best_setup_ms, 4),
              "pcg_ms": round(best_pcg_ms, 4),
              "default_setup_ms": round(next(ms for ms, c in res_setup if not c), 4),
              "default_pcg_ms": round(next(ms for ms, c in res_pcg if not c), 4)}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        store[key] = choice
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(store, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return choice
