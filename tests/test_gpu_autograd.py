"""The torch.autograd wrapper of the compliance adjoint, through the C ABI.

Its forward replaces the geometry on the device (lbddc_set_geometry_device)
and re-solves; its backward contracts the incoming gradient with the
library's adjoint.  Checked against a second context that receives the same
geometry through the host entry point (set_problem) and returns its adjoint
through lbddc_compliance_gradient, and, for the second geometry, against the
oracle's FP64 adjoint."""
import numpy as np
import pytest

from conftest import oracle_roms
from workloads import make_problem

pytestmark = pytest.mark.gpu


def _host_reference(prob, roms, rtol):
    from gpu_helpers import make_solver
    s = make_solver(prob, roms)
    s.assemble()
    s.setup()
    s.solve(rtol=rtol, max_iter=1000)
    out = s.compliance_gradient()
    s.close()
    return out


@pytest.mark.parametrize("cfg,over", [(4, dict(nx=3, ny=3, p=4)), (5, dict(nx=3, ny=2, p=4, nrhs=2))])
def test_compliance_autograd(cfg, over):
    import torch
    from gpu_helpers import rom_arrays, rel
    from paper_2604_09113_amd import lbddc
    from paper_2604_09113_amd.autograd import compliance
    prob = make_problem(cfg, **over)
    roms = oracle_roms(prob)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    s = lbddc.Solver(0, stream.cuda_stream)
    for rom in roms.values():
        s.load_rom(**rom_arrays(rom))
    s.set_problem(prob["nx"], prob["ny"], prob["p"], prob["q"], prob["m"], prob["ctrl"], prob["family"], prob["t"],
                  prob["E"], prob["nu"], prob["rho"], prob["moments"], prob["traction"])
    rng = np.random.default_rng(7)
    # a second geometry: interior net points moved, thicknesses shifted, still inside the ROM box
    ctrl2 = prob["ctrl"].copy()
    ctrl2[1:-1, 1:-1] += 0.01 * rng.normal(size=ctrl2[1:-1, 1:-1].shape)
    t2 = np.clip(prob["t"] + 0.01 * rng.normal(size=prob["t"].shape), 0.11, 0.29)
    for ctrl_h, t_h in ((prob["ctrl"], prob["t"]), (ctrl2, t2)):
        ctrl = torch.tensor(ctrl_h, dtype=torch.float64, device="cuda", requires_grad=True)
        t = torch.tensor(t_h, dtype=torch.float64, device="cuda", requires_grad=True)
        J = compliance(ctrl, t, s, lbddc.FP64, 1e-12)
        w = torch.tensor(rng.normal(size=J.shape[0]), dtype=torch.float64, device="cuda")
        (w * J).sum().backward()
        pr = dict(prob, ctrl=ctrl_h, t=t_h)
        Jr, gXr, gtr = _host_reference(pr, roms, 1e-12)
        wh = w.cpu().numpy()
        eJ = rel(J.detach().cpu().numpy(), Jr)
        eX = rel(ctrl.grad.cpu().numpy(), np.tensordot(wh, gXr, axes=1))
        et = rel(t.grad.cpu().numpy(), np.tensordot(wh, gtr, axes=1))
        print(f"[autograd cfg{cfg}] J {J.detach().cpu().numpy()} rel err J {eJ:.2e} dctrl {eX:.2e} dt {et:.2e}")
        assert eJ <= 1e-12 and eX <= 1e-10 and et <= 1e-10
    # the device-set geometry equals the host-set one: the oracle's adjoint at ctrl2, t2
    from oracle.adjoint import compliance_gradient
    from oracle.bddc import Problem
    P = Problem(dict(prob, ctrl=ctrl2, t=t2), roms)
    P.setup()
    Jo, gXo, gto = compliance_gradient(P, P.direct_solve())
    assert rel(J.detach().cpu().numpy(), Jo) <= 1e-10
    assert rel(ctrl.grad.cpu().numpy(), np.tensordot(wh, gXo, axes=1)) <= 1e-8
    s.close()
    torch.cuda.set_stream(torch.cuda.default_stream())


def test_compliance_refuses_other_stream():
    """A solver whose stream is not the current torch stream is refused."""
    import torch
    from gpu_helpers import make_solver
    from paper_2604_09113_amd.autograd import compliance
    prob = make_problem(4, nx=2, ny=2, p=3)
    s = make_solver(prob, oracle_roms(prob))   # the library's own stream
    ctrl = torch.tensor(prob["ctrl"], dtype=torch.float64, device="cuda", requires_grad=True)
    t = torch.tensor(prob["t"], dtype=torch.float64, device="cuda", requires_grad=True)
    with pytest.raises(ValueError):
        compliance(ctrl, t, s)
    s.close()
