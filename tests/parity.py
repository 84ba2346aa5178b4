"""Comparison helpers shared by the GPU parity tests (no arithmetic of the
method: only the rules for comparing two runs)."""
import numpy as np


def first_near_tie(ev, tie):
    idx = np.nonzero(ev["margin"] <= tie)[0]
    return int(idx[0]) if len(idx) else len(ev)


def compare_events(ev_o, ev_g, tie, key="inc"):
    """Events before the first near-tie (in either run) must be identical.
    Returns the increment (key="inc") or the step (key="step", for runs
    without increments) from which the runs may legitimately diverge, and
    the number of identical events."""
    k = min(first_near_tie(ev_o, tie), first_near_tie(ev_g, tie))
    ko = [(int(e["inc"]), int(e["step"]), int(e["id"])) for e in ev_o[:k]]
    kg = [(int(e["inc"]), int(e["step"]), int(e["id"])) for e in ev_g[:k]]
    assert ko == kg, _first_diff(ko, kg)
    div = 1 << 30
    # the first event past the identical prefix in either list (a list that
    # ran out before the tie must not hide an extra event in the other)
    if k < len(ev_o):
        div = min(div, int(ev_o[k][key]))
    if k < len(ev_g):
        div = min(div, int(ev_g[k][key]))
    return div, k


def compare_trace(rec_o, rec_g, rtol, upto_step=None, dim=2):
    """Records of a constant-rate run (one per callback): the strain exactly,
    sigma_xx, potential and kinetic energy within rtol of max(|value|, 1e-3
    of the run's largest), broken-spring counts equal, for the callbacks
    before step upto_step.  Returns the number compared."""
    peak = {q: max(abs(f(r)) for r in rec_o) or 1.0
            for q, f in (("sxx", lambda r: r["sigma"][0, 0]), ("pe", lambda r: r["pe"]),
                         ("ke", lambda r: r["ke"]))}
    n = 0
    for ro, rg in zip(rec_o, rec_g):
        if upto_step is not None and ro["step"] >= upto_step:
            break
        assert ro["step"] == rg["step"] and ro["inc"] == rg["inc"]
        assert rg["eps"] == ro["eps"], f"step {ro['step']}: strain {rg['eps']!r} vs {ro['eps']!r}"
        for q, vo, vg in (("sxx", ro["sigma"][0, 0], rg["sigma"][0, 0]), ("pe", ro["pe"], rg["pe"]),
                          ("ke", ro["ke"], rg["ke"])):
            scale = max(abs(vo), 1e-3 * peak[q])
            assert abs(vg - vo) <= rtol * scale, f"step {ro['step']}: {q} {vo!r} vs {vg!r}"
        so, sg = ro["sigma"][:dim, :dim], rg["sigma"][:dim, :dim]
        assert np.max(np.abs(sg - so)) <= rtol * max(np.max(np.abs(so)), 1e-3 * peak["sxx"])
        assert rg["n_broken"] == ro["n_broken"], f"step {ro['step']}"
        n += 1
    return n


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


def first_set_difference(ev_a, ev_b, n_inc):
    """First increment after which the sets of springs broken so far differ
    between two runs (n_inc + 1 if they never do); a spring breaks once, so
    the sets agree through increment n iff every increment's own set does."""
    for n in range(1, n_inc + 1):
        a = np.sort(ev_a["id"][ev_a["inc"] == n])
        b = np.sort(ev_b["id"][ev_b["inc"] == n])
        if not np.array_equal(a, b):
            return n
    return n_inc + 1
