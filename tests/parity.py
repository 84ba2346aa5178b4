"""Comparison helpers shared by the GPU parity tests (no arithmetic of the
method: only the rules for comparing two runs)."""
import numpy as np


def first_near_tie(ev, tie):
    idx = np.nonzero(ev["margin"] <= tie)[0]
    return int(idx[0]) if len(idx) else len(ev)


def compare_events(ev_o, ev_g, tie):
    """Events before the first near-tie (in either run) must be identical.
    Returns the increment from which the runs may legitimately diverge."""
    k = min(first_near_tie(ev_o, tie), first_near_tie(ev_g, tie))
    ko = [(int(e["inc"]), int(e["step"]), int(e["id"])) for e in ev_o[:k]]
    kg = [(int(e["inc"]), int(e["step"]), int(e["id"])) for e in ev_g[:k]]
    assert ko == kg, _first_diff(ko, kg)
    div_inc = 1 << 30
    if k < len(ev_o):
        div_inc = min(div_inc, int(ev_o[k]["inc"]))
    if k < len(ev_g):
        div_inc = min(div_inc, int(ev_g[k]["inc"]))
    if k == len(ev_o) and k == len(ev_g):
        return div_inc, k
    # a list that ran out before the tie must not hide an extra event
    if k == len(ev_o) and k < len(ev_g):
        div_inc = min(div_inc, int(ev_g[k]["inc"]))
    if k == len(ev_g) and k < len(ev_o):
        div_inc = min(div_inc, int(ev_o[k]["inc"]))
    return div_inc, k


def _first_diff(a, b):
    for i, (x, y) in enumerate(zip(a, b)):
        if x != y:
            return f"event {i}: oracle {x} gpu {y}"
    return f"lengths {len(a)} vs {len(b)}"


def compare_records(rec_o, rec_g, rtol, dim, upto_inc=None):
    """Stress (Eq. 7) per increment within rtol of max(|sigma|, 1e-3 peak)."""
    peak = max(abs(r["sigma"][0, 0]) for r in rec_o) or 1.0
    pe_peak = max(abs(r["pe"]) for r in rec_o) or 1.0
    n = 0
    for ro, rg in zip(rec_o, rec_g):
        if upto_inc is not None and ro["inc"] >= upto_inc:
            break
        assert ro["inc"] == rg["inc"]
        assert rg["eps"] == ro["eps"]
        so, sg = ro["sigma"][:dim, :dim], rg["sigma"][:dim, :dim]
        # the stress-strain curve (sigma_xx) elementwise, the whole tensor
        # normwise (its largest entry sets the scale of the small ones)
        sxx_scale = max(abs(so[0, 0]), 1e-3 * peak)
        err_xx = abs(sg[0, 0] - so[0, 0]) / sxx_scale
        assert err_xx <= rtol, f"inc {ro['inc']}: sigma_xx rel err {err_xx:.3e}"
        t_scale = max(np.max(np.abs(so)), 1e-3 * peak)
        err = np.max(np.abs(sg - so)) / t_scale
        assert err <= rtol, f"inc {ro['inc']}: sigma rel err {err:.3e}\n{so}\n{sg}"
        assert abs(rg["pe"] - ro["pe"]) <= rtol * max(abs(ro["pe"]), 1e-3 * pe_peak), \
            f"inc {ro['inc']}: pe {ro['pe']} vs {rg['pe']}"
        assert rg["n_broken"] == ro["n_broken"]
        n += 1
    return n
