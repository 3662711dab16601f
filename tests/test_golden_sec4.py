"""The numbers Sec. IV prints (tests/golden/sec4_printed_values.json) against
what the theory tools and the run recipes use.

* the binary critical points follow from Eq. (lgf) exactly (theory tools);
* the quoted ternary critical points are not the plait points of Eq. (lgf)
  (reading R16): they differ by 0.01 to 0.06;
* the run recipes of the Sec. IV experiments use the printed parameters."""
import json
import os

import numpy as np

import lbinputs as LI
from oracle import theory as T

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sec4_printed_values.json")))


def val(key):
    return GOLD[key]["value"]


def test_binary_critical_points_from_the_free_energy():
    for mkey, ckey in (("binary_monomer_m", "binary_monomer_critical_phi"),
                       ("binary_polymer_m", "binary_polymer_critical_phi")):
        mA, mB = val(mkey)
        phi_c, _ = T.binary_critical(mA, mB)
        digits = GOLD[ckey].get("digits", 12)
        assert round(phi_c, digits) == val(ckey)[0] and round(1 - phi_c, digits) == val(ckey)[1]


def test_quoted_ternary_critical_points_vs_plait_points():
    c = val("ternary_chi")
    chi = np.array([[0, c["AB"], c["AC"]], [c["AB"], 0, c["BC"]], [c["AC"], c["BC"], 0]])
    for m, key in (((1, 1, 1), "ternary_monomer_critical_quoted"), ((10, 1, 1), "ternary_polymer_critical_quoted")):
        q = np.array(val(key))
        p = T.ternary_plait_point(m, chi, q)
        assert abs(q.sum() - 1) < 1e-12
        assert 0.01 < np.abs(p - q).max() < 0.06, (key, p)


def test_run_recipes_use_the_printed_parameters():
    mono = LI.binodal_runs("binary_monomer")
    assert sorted({round(1 / r[0]["tau"], 6) for r in mono}) == val("binary_inv_tau_monomer")
    for cfg, rho0, _ in mono[:3]:
        phi = rho0[0] / rho0.sum(axis=0)
        assert abs(phi.mean() - val("binary_monomer_critical_phi")[0]) < 1e-6
        assert abs(0.5 * np.ptp(phi) - val("sine_amplitude")) < 1e-3
    poly = LI.binodal_runs("binary_polymer")
    assert {tuple(r[0]["m"]) for r in poly} == {tuple(float(x) for x in val("binary_polymer_m"))}
    assert {round(1 / r[0]["tau"], 6) for r in poly} == {val("binary_inv_tau_polymer")}
    c = val("ternary_chi")
    for exp, key in (("ternary_monomer", "ternary_monomer_critical_quoted"),
                     ("ternary_polymer", "ternary_polymer_critical_quoted")):
        runs = LI.binodal_runs(exp)
        cfg = runs[0][0]
        assert cfg["chi"][0, 1] == c["AB"] and cfg["chi"][0, 2] == c["AC"] and cfg["chi"][1, 2] == c["BC"]
        assert round(1 / cfg["tau"], 6) == val("ternary_inv_tau")
        # starts on the segment from the quoted critical point to the end point
        start = np.array(val(key))
        end = np.array(val("ternary_segment_end"))
        for cfg_k, rho0, label in runs:
            s = float(label.split("=")[1])
            mean = rho0.mean(axis=1)
            assert np.abs(mean - (start + s * (end - start))).max() < 1e-6, (exp, label)
    cfg2, _ = LI.profile_run("binary_polymer_profile")
    assert cfg2["chi"][0, 1] == val("fig2_chi")
    cfg4, rho4 = LI.profile_run("ternary_polymer_profile")
    assert np.abs(rho4.mean(axis=1) - np.array(val("ternary_polymer_critical_quoted"))).max() < 1e-6
