"""Timing autotuner for the launch shape of the row kernels (batching form).

Every CSR row kernel of the library gives a row of its block width / cpt lanes,
each lane cpt consecutive columns.  Which cpt is fastest depends on the level
(rows, nonzeros per row, how much of the gathered block stays in cache), the
block width and the precision, so it is chosen per (kind, level) by timing the
candidates on the bound context: the V-cycle kernels of a level, the FP64
kernels of the correction level (outer residual, dual SpMM, prolongation, final
update) and the
FP64 restriction of [A V | M V].  The winner must beat the built-in choice by a
margin, otherwise the built-in choice stays.  Results go to an on-disk JSON
cache keyed by device architecture, precision, smoother, kind, level size,
nonzeros and width, so a later context of the same shape is configured without
timing.  The choice never changes the iterates (each vector entry is the same
ordered sum for every cpt); only the residual norms can differ in the last
bits, through the order of their row sums.
"""
import json
import os
import tempfile

from . import PREC_MIXED, TUNE_FP64, TUNE_FP64_WIDE, TUNE_VCYCLE

KINDS = {TUNE_VCYCLE: "vcycle", TUNE_FP64: "fp64", TUNE_FP64_WIDE: "fp64_wide"}


def default_cache_path():
    return os.environ.get("AMG_EIG_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "amg_eig", "cpt_tuning.json"))


def candidates(width):
    return [c for c in (2, 4, 8) if width % c == 0 and width // c <= 64]


def _arch():
    try:
        import torch
        return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gpu").split(":")[0]
    except Exception:
        return "gpu"


def _load(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _save(path, table):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".cpt_tuning.")
    with os.fdopen(fd, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def plan(ctx):
    """(kind, level, width, key fields) for every tunable row-kernel group."""
    info = ctx.info()
    qe, dims = info["qe"], info["dims"]
    nl = len(dims)
    prec = "mixed" if ctx.opts.precision == PREC_MIXED else "fp64"
    out = []
    for level in range(nl - 1):
        nnz = ctx.level_nnz(level)
        for kind in (TUNE_VCYCLE, TUNE_FP64, TUNE_FP64_WIDE):
            if kind == TUNE_FP64_WIDE and level < 1:
                continue
            width = 2 * qe if kind == TUNE_FP64_WIDE else qe
            key = "%s|%s|smoother%d|%s|n%d|nnz%d|w%d" % (_arch(), prec, ctx.opts.smoother, KINDS[kind],
                                                      int(dims[level]), nnz, width)
            out.append((kind, level, width, key))
    return out


def tune(ctx, cache_path=None, reps=10, margin=0.03, use_cache=True):
    """Choose and set cpt for every (kind, level) of a bound context.

    Returns {key: {"kind", "level", "cpt", "us": {cpt: microseconds} or None}}.
    Timing clears the solve state: call init() afterwards."""
    path = cache_path or default_cache_path()
    cache = _load(path) if use_cache else {}
    report = {}
    timed = False
    for kind, level, width, key in plan(ctx):
        if key in cache and cache[key] in candidates(width):
            ctx.set_cpt(kind, level, cache[key])
            report[key] = {"kind": KINDS[kind], "level": level, "cpt": cache[key], "us": None}
            continue
        ctx.set_cpt(kind, level, 0)
        builtin = ctx.get_cpt(kind, level)
        us = {c: ctx.tune_time(kind, level, c, reps) for c in candidates(width)}
        timed = True
        best = min(us, key=lambda c: (us[c], c != builtin))
        if us[best] > (1.0 - margin) * us[builtin]:
            best = builtin
        ctx.set_cpt(kind, level, best)
        cache[key] = best
        report[key] = {"kind": KINDS[kind], "level": level, "cpt": best, "us": us}
    if timed and use_cache:
        _save(path, cache)
    return report
