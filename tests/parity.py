"""Comparison of a renderer's per-ray output with the oracle's.

Bars (written here once, used by every parity test):
  max             bit-exact (-inf for rays that miss the box)
  cell sequences  bit-exact: identity, order and count
  sum             |got - ref| <= 2e-6 |ref|; rays with ref == 0 must give 0
  wmean           |got - ref| <= 2e-6 max(|ref|, A) with A the weighted mean of
                  the summed magnitudes of the terms of f (the line-of-sight
                  mean velocity can be ~0 while its terms are not); weight
                  plane sum(w chord) within 2e-6 relative.  The error under
                  the narrower scale max(|ref|, weighted mean of |f|) is
                  reported beside it (wmean_err_absdot).
"""
import numpy as np

import oracle

REL = 2e-6


def check_sum(got, ref, what=""):
    got = np.asarray(got, np.float64)
    zero = ref == 0.0
    assert np.all(got[zero] == 0.0), f"{what}: rays missing the box must give exactly 0"
    rel = np.abs(got[~zero] - ref[~zero]) / np.abs(ref[~zero])
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= REL, f"{what}: max rel err {worst:.3e} > {REL}"
    return worst


def check_max(got, ref, what=""):
    got = np.asarray(got, np.float32)
    bad = np.nonzero(got.view(np.int32) != ref.view(np.int32))[0]
    assert bad.size == 0, f"{what}: {bad.size} max values differ, first at {bad[:5]}: {got[bad[:5]]} vs {ref[bad[:5]]}"


def wmean_err_absdot(got, ref):
    """Largest |got - ref| / max(|ref|, weighted mean of |f|) over rays with
    weight (reported, not a bar)."""
    got = np.asarray(got, np.float64)
    hit = ref["aux"] > 0
    norm = np.maximum(np.abs(ref["val"]), ref["absdot"])[hit]
    err = np.abs(got[hit] - ref["val"][hit]) / np.where(norm > 0, norm, 1.0)
    return float(err.max()) if err.size else 0.0


def check_wmean(got, aux, ref, what=""):
    got = np.asarray(got, np.float64)
    norm = np.maximum(np.abs(ref["val"]), ref["absf"])
    hit = ref["aux"] > 0
    assert np.all(got[~hit] == 0.0), f"{what}: zero-weight rays must give 0"
    err = np.abs(got[hit] - ref["val"][hit]) / norm[hit]
    worst = float(err.max()) if err.size else 0.0
    assert worst <= REL, f"{what}: wmean err {worst:.3e} > {REL}"
    if aux is not None:
        check_sum(aux, ref["aux"], what + " weight")
    print(f"{what}: wmean err {worst:.3e} (scale A), {wmean_err_absdot(got, ref):.3e} (scale |f|)", flush=True)
    return worst


def check_counts(got, ref, what=""):
    got = np.asarray(got)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, f"{what}: {bad.size} rays differ in cell count, first {bad[:5]}"


def check_trace(offs, cells, ref_offs, ref_cells, what=""):
    assert np.array_equal(np.asarray(offs), ref_offs), f"{what}: per-ray cell counts differ"
    assert np.array_equal(np.asarray(cells), ref_cells), f"{what}: cell sequences differ"


def compare_all(rend, OT, camd, ops=("sum", "max"), rays=None, los_fields=None, trace_rays=None, what=""):
    """rend: object with camera(d), render(cam, op, field, weight, los, rays) -> (out, aux, counts),
    trace(cam, rays).  Renders the requested ops and compares with oracle tree OT."""
    cam = rend.camera(camd)
    ocam = OT.camera(camd)
    assert cam.as_dict() == ocam.as_dict()
    res = {}
    if "sum" in ops:
        out, _, cnt = rend.render(cam, oracle.SUM, rays=rays)
        ref = OT.render(ocam, oracle.SUM, rays=rays)
        res["sum"] = check_sum(out, ref["val"], what + " sum")
        if cnt is not None:
            check_counts(cnt, ref["count"], what + " counts")
    if "max" in ops:
        out, _, _ = rend.render(cam, oracle.MAX, rays=rays)
        check_max(out, OT.render(ocam, oracle.MAX, rays=rays)["max"], what + " max")
    if "wmean" in ops:
        fld, w, los = los_fields
        out, aux, _ = rend.render(cam, oracle.WMEAN, field=fld, weight=w, los=los, rays=rays)
        ref = OT.render(ocam, oracle.WMEAN, field=fld, weight=w, los=los, rays=rays)
        res["wmean"] = check_wmean(out, aux, ref, what + " wmean")
    if trace_rays is not None:
        offs, cells = rend.trace(cam, trace_rays)
        ro, rc, _ = OT.trace(ocam, trace_rays)
        check_trace(offs, cells, ro, rc, what + " trace")
    return res
