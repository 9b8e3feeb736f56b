"""Scheme properties of Sec. 4 on the GPU path (F/D only at fixed
positions, 32^3 jittered lattice, C_v = 1.5 k_B, T = 1): EMS samples the
Gamma law of the internal energies at any time step (distribution error at
the noise floor of ~1.6e6 samples), AMS drifts away from it at large time
steps, and the EMS rejection rate grows like dt^(0.4..0.5)."""
import pytest

pytestmark = pytest.mark.gpu


def test_ems_unbiased_ams_biased_rejection_scaling():
    import numpy as np
    from paper_1707_04232_amd import sdpd
    from paper_1707_04232_amd.studies import fd_only
    print("[case] F/D-only studies", flush=True)
    ems = {dt: fd_only(sdpd.FD_EMS, dt) for dt in (0.05, 1.0, 5.0)}
    ams = fd_only(sdpd.FD_AMS, 5.0)
    for r in ems.values():
        assert r["error_dist"] < 0.015
        assert abs(r["mean_eps_over_CvT"] - 1.0) < 0.005
    assert ams["error_dist"] > 5 * ems[5.0]["error_dist"]
    assert ams["mean_eps_over_CvT"] > 1.03
    x = np.log10(list(ems))
    y = np.log10([r["rejection_rate"] for r in ems.values()])
    slope = np.polyfit(x, y, 1)[0]
    assert 0.3 < slope < 0.6
