"""Launch-shape autotuner for the element kernels.

For a given workload it times the forward (or VJP) element kernel over a grid
of launch shapes -- workgroup size (8 lanes per element, so 8/16/32 elements
per workgroup), persistent-grid depth (waves per CU) and the XCD-aware tile
order -- with the library's own HIP-event kernel timing, keeps the fastest,
applies it with fem_set_launch and caches it in a JSON file keyed by device,
kernel, precision, element variant and a size bucket.  The model variants
(Voce, F-bar, Barlat, a material orientation) run with 64-thread workgroups
whatever the configured size, so for them only the grid depth and the tile
order are searched.

    from paper_2606_17390_amd import tune
    best = tune.tune_forward(mesh, csr, params, d, hist, prec=fem.FP32_MIXED)

The cache path is $FEMHIP_TUNE_CACHE, else ~/.cache/femhip_tune.json.
"""
import json
import math
import os

import torch

from . import fem

BLOCKS = (64, 128, 256)
WAVES = (2, 4, 8, 16)
REMAP = (0, 1)


def cache_path():
    return os.environ.get("FEMHIP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "femhip_tune.json"))


def _launch_prec(prec):
    """The launch slot of a precision (FEM_FP64_K32 runs the FP64 kernels)."""
    p = fem._prec(prec)
    return fem.FP64 if p == fem.FP64_K32 else p


def _variant(params):
    """Element-variant tag of a Params (model flags, orientation)."""
    if params is None:
        return "v0"
    return f"m{params.model}o{1 if params.orient is not None else 0}"


def _key(kernel, prec, n_elems, variant="v0"):
    name = torch.cuda.get_device_name() if torch.cuda.is_available() else "none"
    bucket = int(math.log2(max(n_elems, 1)))
    return f"{name}|k{kernel}|p{_launch_prec(prec)}|{variant}|e2^{bucket}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _time(kernel, fn, reps):
    fn()
    torch.cuda.synchronize()
    fem.timing_read(kernel)
    fem.timing_enable(True)
    try:
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
    finally:
        fem.timing_enable(False)
    ms, n = fem.timing_read(kernel)
    return ms / max(n, 1)


def _search(kernel, prec, fn, reps, blocks, waves, remaps):
    results = []
    try:
        for b in blocks:
            for w in waves:
                for r in remaps:
                    fem.set_launch(kernel, prec, block=b, waves_per_cu=w, xcd_remap=r)
                    results.append((_time(kernel, fn, reps), b, w, r))
    finally:
        fem.set_launch(kernel, prec)
    results.sort()
    return results


def tune(kernel, prec, n_elems, fn, reps=3, blocks=BLOCKS, waves=WAVES, remaps=REMAP, use_cache=True,
         variant="v0"):
    """Tune `fn` (a closure issuing one library call of `kernel`), apply the
    best shape and return (ms, block, waves_per_cu, xcd_remap)."""
    prec = _launch_prec(prec)
    if variant != "v0" and variant != "m0o0":
        blocks = (64,)  # the variant kernels take 64-thread workgroups only
    key = _key(kernel, prec, n_elems, variant)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        ms, b, w, r = db[key]
    else:
        ms, b, w, r = _search(kernel, prec, fn, reps, blocks, waves, remaps)[0]
        if use_cache:
            db[key] = [ms, b, w, r]
            _store(db)
    fem.set_launch(kernel, prec, block=b, waves_per_cu=w, xcd_remap=r)
    return ms, b, w, r


def tune_forward(mesh, csr, params, d, hist, prec=fem.FP32_MIXED, bc_mask=None, batch=None, **kw):
    out = fem.Forward(mesh, csr, prec)

    def fn():
        fem.residual_tangent(mesh, csr, params, d, hist, bc_mask=bc_mask, prec=prec, out=out, batch=batch)
    return tune(fem.KERNEL_FORWARD, prec, mesh.n_elems, fn, variant=_variant(params), **kw)


def tune_vjp(mesh, params, d, hist, lam, prec=fem.FP32_MIXED, batch=None, **kw):
    out = fem.Vjp(mesh, batch.n_spec if batch is not None else 1)

    def fn():
        fem.residual_vjp(mesh, params, d, hist, lam, prec=prec, out=out, batch=batch)
    return tune(fem.KERNEL_VJP, prec, mesh.n_elems, fn, variant=_variant(params), **kw)


def apply_cached(kernel, prec, n_elems, variant="v0"):
    """Apply a cached shape if there is one; returns it or None."""
    db = _load()
    prec = _launch_prec(prec)
    key = _key(kernel, prec, n_elems, variant)
    if key not in db:
        return None
    ms, b, w, r = db[key]
    fem.set_launch(kernel, prec, block=b, waves_per_cu=w, xcd_remap=r)
    return ms, b, w, r
