"""Shared test helpers: masks built independently by the library and the
oracle (and checked byte-equal), and field error norms."""
import numpy as np

import oracle as O


def masks(w, lib=None):
    """Electrode + biofilm-layer mask of workload dict w, built by the oracle
    and (if lib is given) by the library; asserts they are byte-equal."""
    if w["nz"] > 1:
        st, b, _ = O.geom_fibres(w["nx"], w["ny"], w["nz"], w["r_min"], w["r_max"], w["solid"],
                                 w["seed"])
    else:
        st, b, _ = O.geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"],
                                w["overlap"], w["seed"])
    assert st == "OK"
    if w.get("layer", True):
        b = O.biofilm_layer(b)
    if lib is not None:
        if w["nz"] > 1:
            s2, a, _ = lib.lbm_geom_fibres(w["nx"], w["ny"], w["nz"], w["r_min"], w["r_max"],
                                           w["solid"], w["seed"])
        else:
            s2, a, _ = lib.lbm_geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"],
                                          w["overlap"], w["seed"])
        assert s2 == 0
        if w.get("layer", True):
            a = lib.lbm_biofilm_layer(a)
        assert np.array_equal(a, b)
    return b


def rel_l2(got, want, sel=None):
    g = np.asarray(got, np.float64)
    w = np.asarray(want, np.float64)
    if sel is not None:
        g = g[..., sel]
        w = w[..., sel]
    den = np.linalg.norm(w)
    return np.linalg.norm(g - w) / (den if den > 0 else 1.0)


def max_abs(got, want, sel=None):
    g = np.asarray(got, np.float64)
    w = np.asarray(want, np.float64)
    if sel is not None:
        g = g[..., sel]
        w = w[..., sel]
    return float(np.abs(g - w).max()) if g.size else 0.0
