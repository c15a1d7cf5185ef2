"""GPU SCF step (bdg_scf_step) against the CPU oracle step."""
import numpy as np
import pytest

from paper_2310_03341_amd import inputs
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.mark.parametrize("instance", [0, 3, 7])
def test_scf_step_matches_oracle(dev, instance):
    import torch
    from oracle import scf
    from paper_2310_03341_amd import api
    inst = inputs.scf_instance(instance, dims=(16, 16))
    p = inputs.ScfParams()
    ns = inst.Vext.size
    U0 = inst.Vext.copy()
    D0 = np.full(ns, 0.3)
    ref = scf.scf_step(inst.dims, inst.Vext, inst.theta, inst.mu, U0, D0, p)
    st = api.ScfStepper(inst.dims, torch.from_numpy(inst.Vext).to(dev),
                        torch.from_numpy(inst.theta).to(dev), inst.mu, p)
    U = torch.from_numpy(U0.copy()).to(dev)
    D = torch.from_numpy(D0.copy()).to(dev)
    change, m = st.step(U, D)
    torch.cuda.synchronize()
    assert m == ref["m"]
    assert abs(change - ref["change"]) < 1e-10
    assert np.abs(U.cpu().numpy() - ref["U"]).max() < 1e-10
    assert np.abs(D.cpu().numpy() - ref["absDelta"]).max() < 1e-10
    assert np.abs(st.density.cpu().numpy() - ref["n"]).max() < 1e-10
    assert np.abs(st.nu_abs.cpu().numpy() - ref["nu_abs"]).max() < 1e-10


def test_scf_uniform_gas_fixed_point_on_gpu(dev):
    """Uniform gas (no trap, B = 0): the GPU iteration reaches the gap equation."""
    import torch
    from oracle import scf
    from paper_2310_03341_amd import api
    dims = (8, 8)
    p = inputs.ScfParams(B=0.0, alpha=1.0)
    ns = 64
    z = torch.zeros(ns, dtype=torch.float64, device=dev)
    st = api.ScfStepper(dims, z, z, 1.0, p)
    U = torch.zeros(ns, dtype=torch.float64, device=dev)
    D = torch.full((ns,), 0.5, dtype=torch.float64, device=dev)
    for _ in range(200):
        change, m = st.step(U, D)
        if change < 1e-12:
            break
    d = D.cpu().numpy()
    assert np.abs(d - d.mean()).max() < 1e-10
    _, nu = scf.uniform_densities(dims, 0.0, d.mean(), 1.0, p.Ec)
    assert abs(p.g * nu / d.mean() - 1.0) < 1e-9


def test_scf_checkpoint_resume_on_gpu(dev, tmp_path):
    """The SCF iteration on the GPU, interrupted after 7 steps and continued
    from its checkpoint, reaches the iterate of an uninterrupted run of the
    same length (the step is a function of the fields alone)."""
    import torch
    from paper_2310_03341_amd import learned_start as ls
    inst = inputs.scf_instance(3, dims=(12, 12))
    p = inputs.ScfParams(tol=0.0, max_iter=12)
    it_a, _, Ua, Da = ls.solve_instance(inst, p, dev)
    path = str(tmp_path / "scf.npz")
    p7 = inputs.ScfParams(tol=0.0, max_iter=7)
    it_b, ok_b, _, _ = ls.solve_instance(inst, p7, dev, checkpoint=path, every=3)
    assert it_b == 7 and not ok_b
    it_c, _, Uc, Dc = ls.solve_instance(inst, p, dev, checkpoint=path, every=3)
    assert it_a == it_c == 12
    print("max |U - U'| %.2e, max |D - D'| %.2e" % ((Ua - Uc).abs().max().item(), (Da - Dc).abs().max().item()))
    assert torch.allclose(Ua, Uc, rtol=0, atol=1e-12)
    assert torch.allclose(Da, Dc, rtol=0, atol=1e-12)
