"""Config-4 reading (Sec. 4.2 diffuse crack): which crack-moduli floors and
diffuse widths the reflux-free composite cycle of this discretization can
solve.  tests/golden/penny_crack_convergence.json records the oracle's
residual histories (written by tests/golden/penny_crack_convergence.py,
which calls only the oracle and the input generators); these tests check
the record's verdicts and re-run its cheapest cases against the oracle as
it stands, so the record cannot go stale."""
import json
import os

import numpy as np

import synth
from oracle import amr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "penny_crack_convergence.json")


def _runs():
    return {(r["base_nodes"], r["floor"], r["width"]): r for r in json.load(open(GOLDEN))["runs"]}


def test_record_verdicts():
    """Floor 1e-4 (four decades of moduli contrast inside the crack)
    diverges at every width and base; the paper's 1 % cap converges at
    width 0.05 on both bases and at width 0.01 on the 65^3 base (finest
    spacing 1/256, the crack over ~2.6 cells), but not on the 33^3 base."""
    runs = _runs()
    for n in (33, 65):
        for w in (0.01, 0.05):
            r = runs[(n, 1e-4, w)]
            assert r["rel_res"][-1] > 1e3 and r["factor_last10"] > 1.0, (n, w)
    for n in (33, 65):
        r = runs[(n, 1e-2, 0.05)]
        assert r["rel_res"][-1] < 1e-5 and r["factor_last10"] < 0.8, n
    assert runs[(65, 1e-2, 0.01)]["factor_last10"] < 0.85 and runs[(65, 1e-2, 0.01)]["rel_res"][-1] < 1e-4
    assert runs[(33, 1e-2, 0.01)]["rel_res"][-1] > 1e3


def _history(n, floor, width, cycles):
    ap = synth.penny_crack(n=n, levels=3, floor=floor, width=width)
    comp = amr.from_problem(ap)
    u = comp.initial()
    r0 = comp.norm(comp.residual(u))
    out = [1.0]
    for _ in range(cycles):
        u = comp.cycle(u)
        out.append(comp.norm(comp.residual(u)) / r0)
    return ap, out


def test_record_matches_the_oracle_as_it_stands():
    runs = _runs()
    ap, h = _history(33, 1e-4, 0.01, 2)
    rec = runs[(33, 1e-4, 0.01)]
    assert [len(ap.level_boxes(k)) for k in (1, 2)] == rec["boxes_per_level"]
    assert ap.composite_nodes() == rec["composite_nodes"]
    np.testing.assert_allclose(h, rec["rel_res"][:3], rtol=1e-9)
    _, h = _history(33, 1e-2, 0.05, 4)
    np.testing.assert_allclose(h, runs[(33, 1e-2, 0.05)]["rel_res"][:5], rtol=1e-9)
