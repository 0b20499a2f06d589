"""The spurious-current study driver: case set and parameters on the CPU, a
short run of the batched study on the GPU."""
import json
import math

import pytest


def test_case_set_and_parameters():
    from paper_2205_05835_amd import spurious as sp
    cases = sp.build_cases([16, 32, 64], 1.0, "fp64")
    assert len(cases) == 2 * 3 * 9
    pairs = {(c["model"], c["force"]) for c in cases}
    assert len(pairs) == 9
    for c in cases:
        h = 1.0 / c["n"]
        if c["panel"] == "fixed":
            assert c["eps"] == 1.0 / 32.0
        else:   # the refinement path of Sec. 3.1: dx = sqrt(32) eps^(3/2)
            assert math.isclose(h, math.sqrt(32.0) * c["eps"] ** 1.5, rel_tol=1e-12)
        p = c["params"]
        assert p.walls == 3                                 # free-slip walls on all sides (Sec. 3.1)
        assert p.rho1 == p.rho2 == 300.0 and p.visc1 == p.visc2 == 0.1 and p.sigma == 1.0
        # La = sigma rho D / visc^2 = 12000 (Sec. 3.1)
        assert math.isclose(p.sigma * p.rho1 * sp.DIAM / p.visc1 ** 2, 12000.0)
    # the limits of the explicit step at N = 128, eps = 1/32, gamma = 1
    dt = sp.stable_dt(128, 1.0 / 32.0, 1.0)
    assert math.isclose(dt, 0.1 / 128 ** 2 * 32.0)


@pytest.mark.gpu
def test_short_study_on_gpu(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_05835_amd import spurious as sp
    out = tmp_path / "s.json"
    print("spurious-current study, N = 16 and 32, t* to 2", flush=True)
    sp.main(["--n", "16", "32", "--t-end", "2", "--t-sample", "1", "--t-report", "2", "--gamma", "0.01",
             "--out", str(out)])
    d = json.loads(out.read_text())
    assert d["tstar"] == [0.0, 1.0, 2.0]
    assert "walls" in d["setup"]["box"]
    assert len(d["cases"]) == 36
    for c in d["cases"]:
        assert c["ca_inf"][0] == 0.0                       # u = 0 at t = 0
        assert all(math.isfinite(x) and 0.0 < x < 1e-2 for x in c["ca_inf"][1:])
