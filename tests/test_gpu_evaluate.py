"""The evaluation harness end to end on the device (small square-array
scene): complexity, map error and localisation accuracy behave as the
definitions require."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_harness_on_paper_near_field_scene():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08514_amd import evaluate as ev
    print("[gpu-case] evaluate nf4 scene", flush=True)
    res = ev.run("nf4", n_sources=3, frames=4, forms=["fd", "si", "td", "slri", "sspi", "lr"])
    rows = {(r["form"], r["setting"]): r for r in res["rows"]}
    assert res["frames"] == 12 and res["J"] == 73084
    fd = rows[("fd", 0)]
    # four microphones spanning 4 x 5 m: FD places free-field sources within 16 cm
    assert fd["eps_z_db"] is None and fd["rho_s"]["0.16"] >= 0.75
    si = next(r for r in res["rows"] if r["form"] == "si")
    assert si["eps_z_db"]["median"] < -20.0
    assert abs(si["C_rel"] - 0.2456) < 0.01   # Table 1: C_rel(SI) = 0.25 in the NF scenario
    slri = sorted((r for r in res["rows"] if r["form"] == "slri"), key=lambda r: r["setting"])
    c = [r["C_rel"] for r in slri]
    assert c == sorted(c) and all(0 < v < 1 for v in c)
    assert slri[-1]["eps_z_db"]["median"] < slri[0]["eps_z_db"]["median"]
    lr = sorted((r for r in res["rows"] if r["form"] == "lr"), key=lambda r: r["setting"])
    e_h = [r["eps_H_db"] for r in lr]
    assert e_h == sorted(e_h, reverse=True)
    assert lr[-1]["eps_z_db"]["median"] < lr[0]["eps_z_db"]["median"]
    for r in res["rows"]:
        rho = [r["rho_s"][k] for k in ("0.04", "0.08", "0.16")] if "rho_s" in r else []
        assert rho == sorted(rho) and all(0.0 <= v <= 1.0 for v in rho)
    print(ev.markdown(res))
