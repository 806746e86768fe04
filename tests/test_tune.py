"""Launch-shape autotuner: cache handling on the host (CPU) and one small
search on the device (GPU), whose applied shape must leave every output
bitwise unchanged (each entry is summed in a fixed order whatever the shape)."""
import json

import numpy as np
import pytest

from paper_2606_17390_amd import synth


@pytest.fixture
def tune_mod(tmp_path, monkeypatch):
    monkeypatch.setenv("FEMHIP_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_2606_17390_amd import tune
    return tune


def test_cache_round_trip(tune_mod):
    assert tune_mod._load() == {}
    tune_mod._store({"a": [1.0, 64, 4, 1]})
    assert tune_mod._load() == {"a": [1.0, 64, 4, 1]}
    with open(tune_mod.cache_path()) as f:
        assert json.load(f)["a"][1] == 64


def test_key_buckets_by_size(tune_mod):
    from paper_2606_17390_amd import fem
    k1 = tune_mod._key(fem.KERNEL_FORWARD, fem.FP64, 1000)
    k2 = tune_mod._key(fem.KERNEL_FORWARD, fem.FP64, 1023)
    k3 = tune_mod._key(fem.KERNEL_FORWARD, fem.FP64, 4096)
    k4 = tune_mod._key(fem.KERNEL_VJP, fem.FP64, 1000)
    k5 = tune_mod._key(fem.KERNEL_FORWARD, fem.FP32_MIXED, 1000)
    assert k1 == k2 and len({k1, k3, k4, k5}) == 4


def test_apply_cached_sets_the_launch(tune_mod):
    from paper_2606_17390_amd import fem
    assert tune_mod.apply_cached(fem.KERNEL_VJP, fem.FP64, 5000) is None
    key = tune_mod._key(fem.KERNEL_VJP, fem.FP64, 5000)
    tune_mod._store({key: [0.5, 256, 2, 0]})
    try:
        assert tune_mod.apply_cached(fem.KERNEL_VJP, fem.FP64, 5000) == (0.5, 256, 2, 0)
        c = fem.get_launch(fem.KERNEL_VJP, fem.FP64)
        assert (c.block, c.waves_per_cu, c.xcd_remap) == (256, 2, 0)
    finally:
        fem.set_launch(fem.KERNEL_VJP, fem.FP64)


def test_variant_shapes_and_fp64_k32_slot(tune_mod, monkeypatch):
    """A model variant is tuned over 64-thread workgroups only (the only size
    its kernels take), under its own cache key; FEM_FP64_K32 is tuned and set
    in the FP64 launch slot."""
    from paper_2606_17390_amd import fem
    seen = {}

    def fake_search(kernel, prec, fn, reps, blocks, waves, remaps):
        seen.update(blocks=tuple(blocks), prec=prec)
        return [(1.0, blocks[-1], waves[0], remaps[0])]

    monkeypatch.setattr(tune_mod, "_search", fake_search)
    k_plain = tune_mod._key(fem.KERNEL_FORWARD, fem.FP64, 5000)
    k_fbar = tune_mod._key(fem.KERNEL_FORWARD, fem.FP64, 5000, "m2o0")
    assert k_plain != k_fbar
    assert tune_mod._key(fem.KERNEL_FORWARD, fem.FP64_K32, 5000) == k_plain
    try:
        res = tune_mod.tune(fem.KERNEL_FORWARD, fem.FP64_K32, 5000, None, variant="m2o0")
        assert seen["blocks"] == (64,) and seen["prec"] == fem.FP64
        c = fem.get_launch(fem.KERNEL_FORWARD, fem.FP64_K32)
        assert (c.block, c.waves_per_cu, c.xcd_remap) == res[1:]
        c64 = fem.get_launch(fem.KERNEL_FORWARD, fem.FP64)
        assert (c64.block, c64.waves_per_cu, c64.xcd_remap) == res[1:]
        tune_mod.tune(fem.KERNEL_FORWARD, fem.FP64, 5000, None, variant="m0o0", use_cache=False)
        assert seen["blocks"] == tune_mod.BLOCKS
    finally:
        fem.set_launch(fem.KERNEL_FORWARD, fem.FP64)


@pytest.mark.gpu
def test_tune_forward_applies_a_shape_and_keeps_results(tune_mod):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2606_17390_amd import fem
    p = synth.small_slab(44, 13, 5, 3)
    mesh = fem.Mesh(p.X, p.conn)
    params = fem.Params(p.prm, p.n_elems)
    d = torch.as_tensor(p.d).cuda()
    h = torch.as_tensor(p.hist_n).cuda()
    bc = torch.as_tensor(p.bc_mask).cuda()
    csr = fem.csr_pattern(mesh)
    print("tune: forward fp32-mixed on small_slab 13x5x3", flush=True)
    try:
        fem.set_launch(fem.KERNEL_FORWARD, fem.FP32_MIXED)
        ref = fem.residual_tangent(mesh, csr, params, d, h, bc_mask=bc, prec=fem.FP32_MIXED)
        torch.cuda.synchronize()
        ms, b, w, r = tune_mod.tune_forward(mesh, csr, params, d, h, prec=fem.FP32_MIXED, bc_mask=bc, reps=2,
                                            blocks=(64, 128), waves=(2, 8), remaps=(0, 1))
        assert ms > 0 and b in (64, 128) and w in (2, 8) and r in (0, 1)
        c = fem.get_launch(fem.KERNEL_FORWARD, fem.FP32_MIXED)
        assert (c.block, c.waves_per_cu, c.xcd_remap) == (b, w, r)
        # a second call is served from the cache
        assert tune_mod.tune_forward(mesh, csr, params, d, h, prec=fem.FP32_MIXED, bc_mask=bc)[1:] == (b, w, r)
        out = fem.residual_tangent(mesh, csr, params, d, h, bc_mask=bc, prec=fem.FP32_MIXED)
        torch.cuda.synchronize()
        for name in ("R", "K", "hist"):
            assert np.array_equal(getattr(out, name).cpu().numpy(), getattr(ref, name).cpu().numpy()), name
    finally:
        fem.set_launch(fem.KERNEL_FORWARD, fem.FP32_MIXED)
