"""The allocation-free entry point agis_chi2_noalloc (its partial sums in a
per-GPU static scratch array) against agis_chi2, through the C ABI: bit for
bit on two calls in a row on one GPU, the second on a smaller problem (fewer
knot intervals, so fewer partial sums than the first call left in the
array), with the result in host and in device memory; a problem with more
knot intervals than the array holds is refused."""
import numpy as np
import pytest

import synth.configs as C
from test_gpu_parity import agis_mod  # noqa: F401

pytestmark = pytest.mark.gpu


def _loaded(agis, oracle_lib, name):
    w = C.make(name)
    eta = oracle_lib.observed_field_angles(w)
    ctx = agis.agis_create(w.consts, w.knots)
    agis.agis_load_observations(ctx, w.t, eta, w.sigma, w.src, w.fov, w.cell, w.src_true.shape[0], w.n_cells)
    agis.agis_set_sources(ctx, w.src_start)
    agis.agis_set_attitude(ctx, w.att_start)
    agis.agis_set_calibration(ctx, w.cal_start)
    return w, ctx


def test_chi2_noalloc_equals_chi2(agis_mod, oracle_lib):
    import torch
    n_iv = []
    for name in ("tiny", "small9"):                 # the second has fewer knot intervals
        w, ctx = _loaded(agis_mod, oracle_lib, name)
        n_iv.append(w.knots.size - 7)
        for _ in range(2):
            q_ref = agis_mod.agis_chi2(ctx)
            q_host = agis_mod.agis_chi2_noalloc(ctx)
            q_dev = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            agis_mod.agis_chi2_noalloc(ctx, q_dev)
            print(f"{name}: {n_iv[-1]} knot intervals, chi2 {q_ref!r} (no-alloc host {q_host!r}, "
                  f"device {q_dev.item()!r})")
            assert q_host == q_ref and q_dev.item() == q_ref
            agis_mod.agis_iterate(ctx, 1, stats=False)   # another state for the second round
        agis_mod.agis_destroy(ctx)
    assert n_iv[1] < n_iv[0]


def test_chi2_noalloc_refuses_beyond_its_scratch(agis_mod):
    w = C.make("small9")
    K = 131071 * 64 + 1                               # one interval beyond the 1 MiB array
    inner = np.arange(K + 1, dtype=np.float64)
    knots = np.r_[np.zeros(3), inner, np.full(3, inner[-1])]
    ctx = agis_mod.agis_create(w.consts, knots)
    e = np.zeros(0)
    agis_mod.agis_load_observations(ctx, e, e, e.astype(np.float32), e.astype(np.int32), e.astype(np.int8),
                                    e.astype(np.int32), 1, 2)
    with pytest.raises(agis_mod.AgisError) as err:
        agis_mod.agis_chi2_noalloc(ctx)
    assert err.value.code == -2
    agis_mod.agis_destroy(ctx)
