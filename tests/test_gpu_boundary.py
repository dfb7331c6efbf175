"""The boundary's device-memory and result rules on the GPU:

* rom_set_allocator: with PyTorch's caching allocator installed (the binding's default on a GPU
  machine) every buffer of a solve is counted by torch.cuda.memory_allocated() and given back at
  rom_destroy; results are bitwise the same with librom's own hipMalloc;
* rom_phi_device: a solve that fails after its arguments were accepted leaves no device result
  behind (the plan that held the previous one may be gone), so the call reports ROM_E_STATE.
"""
import gc

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


def _problem(R, n=64):
    f = RI.uniform_fields(n, n, 1.0, 0.5, 0.45, 0.55)
    h = R.Handle(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q)
    d, w = R.generate_ordinates(R.ROM_ORD_STRATIFIED, 4, 8, seed=3)
    h.set_ordinates(d, w)
    return f, h, d, w


def test_torch_allocator_holds_librom_memory(R, orc):
    import torch
    R.use_torch_allocator()
    gc.collect()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    f, h, d, w = _problem(R)
    o = R.si_opts(tol=1e-6, tile=(8, 8), band=2, sweep=R.ROM_SWEEP_STRIP)
    phi, st, rc = h.source_iterate(o)
    assert rc == 0
    held = torch.cuda.memory_allocated() - base
    # at least the FP32 fields, flux, source and partial-flux planes of the 64 x 64 problem
    assert held >= 6 * f.cells * 4, held
    ref = orc.source_iterate(orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q), d, w, None, tol=1e-6)
    parity.si_check(orc, orc.Problem(f.nx, f.ny, f.sigma_t, f.sigma_s, f.q), d, w, None, phi, st.iters, 1e-6,
                    1e-5, ref=ref)
    mean, var, est, rc = h.ensemble(4, 9, R.ROM_ORD_STRATIFIED, 2, 2, o)
    assert rc == 0
    assert torch.cuda.memory_allocated() - base > held  # the ensemble's plan and moments
    h.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_hip_allocator_gives_identical_results(R):
    import torch
    o = R.si_opts(tol=1e-6, tile=(8, 8), band=2, sweep=R.ROM_SWEEP_STRIP)
    R.use_torch_allocator()
    _, h1, _, _ = _problem(R)
    phi_t, st_t, _ = h1.source_iterate(o)
    R.use_hip_allocator()
    try:
        gc.collect()
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        _, h2, _, _ = _problem(R)
        phi_h, st_h, _ = h2.source_iterate(o)
        assert torch.cuda.memory_allocated() == base  # hipMalloc: nothing through torch
        assert st_h.iters == st_t.iters and np.array_equal(phi_h, phi_t)
        h2.close()
    finally:
        R.use_torch_allocator()
    # a block taken from torch before the switch is still returned to torch
    h1.close()


def test_failed_solve_leaves_no_device_result(R):
    _, h, _, _ = _problem(R, 32)
    phi, st, rc = h.source_iterate(R.si_opts(tol=1e-6))
    assert rc == 0
    dev, f64 = h.phi_device()
    assert dev and not f64
    # accepted by the argument check, refused while the plan is built (FP64 takes 8 x 4 and
    # 8 x 8 tiles only): the cached plan that held the previous result is released
    with pytest.raises(R.RomError) as e:
        h.source_iterate(R.si_opts(tol=1e-6, precision=R.ROM_PREC_FP64, tile=(16, 16), sweep=R.ROM_SWEEP_STRIP))
    assert e.value.status == R.ROM_E_ARG
    with pytest.raises(R.RomError) as e:
        h.phi_device()
    assert e.value.status == R.ROM_E_STATE
    # a new solve gives a new result
    phi2, _, rc = h.source_iterate(R.si_opts(tol=1e-6))
    assert rc == 0 and np.array_equal(h.phi_device_tensor().cpu().numpy().astype(np.float64), phi2)
    # an ensemble's result is its mean; the per-sample call that follows leaves none
    mean, var, st, rc = h.ensemble(3, 1, R.ROM_ORD_STRATIFIED, 2, 2, R.si_opts(tol=1e-6))
    assert rc == 0
    t = h.phi_device_tensor()
    assert np.array_equal(t.cpu().numpy(), mean)
    h.ensemble_samples(2, 1, R.ROM_ORD_STRATIFIED, 2, 2)
    with pytest.raises(R.RomError) as e:
        h.phi_device()
    assert e.value.status == R.ROM_E_STATE
