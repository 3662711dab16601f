"""Host-side reading of coexisting phases from a line profile
(paper_0704_3444_amd.phase), on hand-made profiles."""
import numpy as np

from paper_0704_3444_amd.phase import _domains, coexisting_phases


def test_domains_of_a_periodic_line():
    m = np.array([1, 1, 0, 0, 1, 0, 1, 1], dtype=bool)
    # the run at the end wraps into the run at the start
    assert sorted(_domains(m)) == [(4, 1), (6, 4)]
    assert _domains(np.ones(5, bool)) == [(0, 5)]
    assert _domains(np.zeros(5, bool)) == []


def test_coexisting_phases_of_flat_plateaus():
    L = 128
    x = np.arange(L)
    # two A-rich domains of different widths, tanh interfaces, plateaus 0.9 / 0.2
    prof = np.zeros(L)
    for lo, hi in ((10, 60), (80, 100)):
        prof += 0.5 * (np.tanh((x - lo) / 1.5) - np.tanh((x - hi) / 1.5))
    phiA = 0.2 + 0.7 * prof
    rho = np.stack([phiA * 2.0, (1 - phiA) * 2.0])  # total density 2: phi is what counts
    res = coexisting_phases(rho)
    assert res["domains"] == 2
    assert abs(res["rich"][0] - 0.9) < 1e-9 and abs(res["poor"][0] - 0.2) < 1e-6
    assert np.allclose(res["rich"].sum(), 1.0) and np.allclose(res["poor"].sum(), 1.0)
    assert res["spread"] < 1e-5


def test_no_separation_and_unflat_plateau():
    L = 64
    rho = np.stack([np.full(L, 0.5) + 0.001 * np.sin(np.arange(L)), np.full(L, 0.5)])
    assert coexisting_phases(rho) is None
    x = np.arange(L)
    phiA = np.where((x >= 16) & (x < 48), 0.8 + 0.05 * np.sin(np.pi * (x - 16) / 32), 0.3)
    res = coexisting_phases(np.stack([phiA, 1 - phiA]))
    assert 0.01 < res["spread"] < 0.02
