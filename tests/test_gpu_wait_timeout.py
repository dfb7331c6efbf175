"""The time-out path of the sweeps' dependency waits, forced from the host.

Every wait between wavefronts (strip edges, LDS rings, band progress counters) is bounded by a
poll count and by the device clock, records an error when it gives up, and lets every other
wave leave its waits; the host then reports ROM_E_DEVICE.  ROM_SPIN_LIMIT=1 makes any wait that
has to poll give up at once: the solve must come back with ROM_E_DEVICE in well under the clock
bound (2 s per wait), no kernel may hang, and a fresh handle afterwards must solve correctly."""
import os
import time

import numpy as np
import pytest

import parity
import rom_inputs as RI

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12527_amd import rom
    rom.lib()
    return rom


@pytest.mark.parametrize("kind", ["strip", "diag"])
def test_forced_wait_timeout_reports_device_error(R, orc, kind):
    f = RI.uniform_fields(256, 256, 1.0, 0.5, 0.45, 0.55)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 4, 4, seed=2)
    if kind == "strip":
        o = R.si_opts(tol=1e-6, tile=(8, 4), band=2, sweep=R.ROM_SWEEP_STRIP)
    else:
        o = R.si_opts(tol=1e-6, sweep=R.ROM_SWEEP_DIAG, diag_rows=16, diag_k=1, band=4)
    os.environ["ROM_SPIN_LIMIT"] = "1"
    try:
        h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
        h.set_ordinates(d, w)
        t0 = time.perf_counter()
        with pytest.raises(R.RomError) as e:
            h.source_iterate(o)
        elapsed = time.perf_counter() - t0
        assert e.value.status == R.ROM_E_DEVICE
        assert elapsed < 30.0, elapsed
        h.close()
    finally:
        del os.environ["ROM_SPIN_LIMIT"]
    # the device is fine: a new handle (its plan built with the normal bounds) solves correctly
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    h.set_ordinates(d, w)
    phi, st, rc = h.source_iterate(o)
    assert rc == 0
    p = orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    parity.si_check(orc, p, d, w, None, phi, st.iters, 1e-6, 1e-5)
