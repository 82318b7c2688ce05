"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and its host
logic (level table, parameter layout, validation) agrees with the oracle.  No GPU calls."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2506_19742_amd import nic, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "nic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nic_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = nic.lib()
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(nic.EXPORTS) == declared


@pytest.mark.parametrize("wname", ["tiny64", "ct256", "ct512"])
def test_level_table_matches_oracle(ora, wname):
    w = synth.WORKLOADS[wname]
    cfg = nic.config_for(w, precision=0)
    lay = nic.nic_describe(cfg)
    ocfg = ora.Config(w.n_levels, w.feats, w.log2_table, w.base_res, w.max_res, w.depth, w.width)
    res, dense, off, size, n = ora.levels(ocfg)
    assert lay["res"] == res.tolist()
    assert lay["dense"] == dense.tolist()
    assert lay["offset"] == off.tolist()
    assert lay["n_entries"] == n
    tot, nt, nd = ora.n_params(ocfg)
    assert lay["n_table"] == nt and lay["n_dense"] == nd
    assert lay["dense_offset"] >= nt and lay["dense_offset"] % 64 == 0
    assert lay["n_params_padded"] >= lay["dense_offset"] + nd


def test_paper_scale_sizes():
    """The 256^3 workload: 16 levels (5 dense), 6,098,925 entries, 12,202,171 parameters."""
    lay = nic.nic_describe(nic.config_for(synth.WORKLOADS["ct256"]))
    assert sum(lay["dense"]) == 5
    assert lay["n_entries"] == 6098925
    assert lay["n_table"] + lay["n_dense"] == 12202171


@pytest.mark.parametrize("width", [32, 64])
def test_gradient_bins_cover_all_tables(width):
    """Bins widen (2^bin_shift entries, at least the 2^13 entries of the bin reduction's LDS tile) as
    tables are added so the per-bin histogram stays in LDS."""
    w = synth.WORKLOADS["ct256"]
    prev = 0
    for K in (1, 2, 4, 8, 16, 32):
        lay = nic.nic_describe(nic.config_for(w, n_tables=K, mlp_width=width))
        ent = lay["n_entries"] * K
        assert lay["bin_shift"] >= 12 and lay["bin_shift"] >= prev
        assert lay["n_bins"] == -(-ent // (1 << lay["bin_shift"]))
        assert lay["n_bins"] * 4 <= 160 * 1024
        if lay["bin_shift"] > 12:   # the narrower bins would not have fitted beside the kernels' tiles
            assert -(-ent // (1 << (lay["bin_shift"] - 1))) > lay["n_bins"]
        prev = lay["bin_shift"]
    assert nic.nic_describe(nic.config_for(w, n_tables=1))["bin_shift"] == 13


def test_workspace_size_and_validation():
    g = synth.cone_geometry(64, 50)
    cfg = nic.config_for(synth.WORKLOADS["tiny64"])
    n = nic.nic_workspace_size(cfg, g)
    assert n > 4 * 4 * 236803
    bad = [dict(n_levels=7), dict(feats_per_level=4), dict(samples_per_ray=48), dict(rays_per_step=0),
           dict(rays_per_step=64 * 64 + 1), dict(mlp_width=48), dict(mlp_depth=9), dict(log2_table=40),
           dict(lr=-1.0), dict(beta1=1.0), dict(precision=3), dict(ln_eps=0.0)]
    for over in bad:
        c = nic.config_for(synth.WORKLOADS["tiny64"], **over)
        with pytest.raises(nic.NicError) as ei:
            nic.nic_workspace_size(c, g)
        assert ei.value.status == nic.NIC_EINVAL
        assert nic.lib().nic_last_error().decode()


def test_geometry_validation():
    cfg = nic.config_for(synth.WORKLOADS["tiny64"])
    for over in [dict(dso=100.0), dict(dsd=900.0), dict(du=0.0), dict(nu=0)]:
        g = synth.cone_geometry(64, 50)
        for k, v in over.items():
            setattr(g, k, v)
        with pytest.raises(nic.NicError):
            nic.nic_workspace_size(cfg, g)
    g = synth.cone_geometry(64, 50)
    g.angles = np.array([0.0, float("nan")])
    with pytest.raises(nic.NicError):
        nic.nic_workspace_size(cfg, g)


def test_create_rejects_bad_workspace_without_gpu():
    """Argument errors are reported before any device call."""
    cfg = nic.config_for(synth.WORKLOADS["tiny64"])
    g = nic.geometry_struct(synth.cone_geometry(64, 50))
    h = C.c_void_p()
    st = nic.lib().nic_create(C.byref(cfg.c()), C.byref(g), None, None, 0, C.byref(h))
    assert st == nic.NIC_EINVAL
    st = nic.lib().nic_create(C.byref(cfg.c()), C.byref(g), None, C.c_void_p(256), 16, C.byref(h))
    assert st == nic.NIC_ENOMEM
    st = nic.lib().nic_create(C.byref(cfg.c()), C.byref(g), None, C.c_void_p(1024 + 8), 1 << 40, C.byref(h))
    assert st == nic.NIC_EINVAL
    assert not h.value
