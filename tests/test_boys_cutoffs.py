"""The device Boys function switches, for highest order L, from its tabulated Taylor grid to the asymptotic form
F_m(T) = Gamma(m+1/2) / (2 T^{m+1/2}) at T_L.  The exact F_m is that form times the regularised lower incomplete
gamma P(m+1/2, T), so the relative error of the switch is Q(m+1/2, T) <= Q(L+1/2, T).  Checks the constants in
the device header against that bound (scipy's incomplete gamma) and against the grid's range."""
import os
import re

from scipy.special import gammaincc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _consts():
    h = open(os.path.join(ROOT, "paper_1303_4916_amd", "csrc", "uqc_device_common.h")).read()
    cut = [float(x) for x in re.search(r"kBoysAsymT\[9\] = \{([^}]*)\}", h).group(1).split(",")]
    i = open(os.path.join(ROOT, "paper_1303_4916_amd", "csrc", "uqc_internal.h")).read()
    tmax = int(re.search(r"constexpr int kBoysTmax = (\d+);", i).group(1))
    return cut, tmax


def test_asymptotic_cutoffs_meet_the_bound():
    cut, tmax = _consts()
    assert len(cut) == 9
    for L, T in enumerate(cut):
        assert T <= tmax, (L, T)                           # the grid covers every T below the cut
        for m in range(L + 1):
            assert gammaincc(m + 0.5, T) <= 2e-17, (L, m, T)
        assert gammaincc(L + 0.5, T - 1) > 2e-17 or T == tmax, (L, T)  # no looser than needed
