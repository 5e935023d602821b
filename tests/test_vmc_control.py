"""Host-side control of the SR training loop (Sec. 3.4): the N_skip = 5/r
rule and the halving of dtau when the energy stops decreasing."""
import pytest

from paper_2206_14307_amd.vmc import DtauSchedule, nskip_from_acceptance


def test_nskip_rule():
    assert nskip_from_acceptance(1.0) == 5
    assert nskip_from_acceptance(0.5) == 10
    assert nskip_from_acceptance(0.18) == 28          # ceil(27.8)
    assert nskip_from_acceptance(0.05) == 100         # the paper's typical 30-100
    assert nskip_from_acceptance(0.0) == 1000         # capped
    assert nskip_from_acceptance(10.0) == 1           # at least one proposal


def test_dtau_halves_only_when_a_window_does_not_improve():
    s = DtauSchedule(0.04, window=2, dtau_min=0.01)
    for e in (-1.0, -1.1):
        s.update(e)
    assert s.dtau == 0.04                             # first window: nothing to compare
    for e in (-1.2, -1.3):
        s.update(e)
    assert s.dtau == 0.04                             # improved
    for e in (-1.3, -1.2):
        s.update(e)
    assert s.dtau == 0.02                             # mean -1.25 not below -1.25
    for e in (-1.0, -1.0):
        s.update(e)
    assert s.dtau == 0.01
    for e in (-0.5, -0.5):
        s.update(e)
    assert s.dtau == pytest.approx(0.01)              # floor
