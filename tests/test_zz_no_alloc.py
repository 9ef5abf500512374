"""The allocation-free entry point (sfac_solve_noalloc) against the plan path it varies
(sfac_plan_create + sfac_step + sfac_plan_flags): two calls in a row, the second on a smaller
input, each bitwise equal to a plan's result with the same status; both arithmetics."""
import sys

import numpy as np
import pytest
from conftest import progress

from paper_2209_08437_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    progress(msg)   # past the output capture: long tests show they are alive


def _instance(ns, seed):
    rng = np.random.default_rng(seed)
    inst = W.Instance(ns, tuple(float(a) for a in rng.uniform(1.1, 1.9, len(ns))), float(rng.uniform(0.05, 0.2)),
                      float(rng.uniform(2e-3, 1e-2)), W.mesh_widths(ns), 0)
    inst.u0 = W.uniform_field(inst.shape, -0.95, 0.95, seed=seed)
    return inst


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_solve_matches_plans_on_two_calls(sfac_lib, dtype):
    import torch
    from paper_2209_08437_amd import sfac
    tdt = torch.float64 if dtype == "f64" else torch.float32
    # the larger call first (3D, several kernels), then a smaller one (2D) over the same workspace
    for ns, steps, seed in (((40, 33, 35), 7, 1), ((63, 20), 5, 2)):
        inst = _instance(ns, seed)
        _say(f"case noalloc {dtype} {ns} {steps} steps")
        u = torch.tensor(inst.u0, dtype=tdt, device="cuda")
        flags, vmax = sfac.solve_noalloc(u, inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, steps, dtype)
        ref = torch.tensor(inst.u0, dtype=tdt, device="cuda")
        with sfac.Plan(inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, dtype) as p:
            p.step(ref, steps)
            f_ref, m_ref = p.flags()
        torch.cuda.synchronize()
        assert torch.equal(u, ref), (dtype, ns)
        assert flags == f_ref == 0 and vmax == m_ref and 0 < vmax <= 1.0


def test_noalloc_solve_status_and_limits(sfac_lib):
    """The status words start at zero on every call (a NaN seen by one call is not reported by
    the next), and an instance whose tables do not fit the workspace is refused."""
    import torch
    from paper_2209_08437_amd import sfac
    inst = _instance((31, 17), 3)
    u = torch.tensor(inst.u0, device="cuda")
    u[2, 3] = float("nan")
    flags, _ = sfac.solve_noalloc(u, inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, 2)
    assert flags & sfac.FLAG_NONFINITE
    u = torch.tensor(inst.u0, device="cuda")
    flags, vmax = sfac.solve_noalloc(u, inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, 2)
    assert flags == 0 and 0 < vmax <= 1.0
    # three axes of N = 2048 (transform length 4096 each) need 576 KiB of tables: refused before
    # the state is touched (a one-element buffer stands in for the 8.6e9-point state)
    import ctypes
    L = sfac.lib()
    ns = (2048, 2048, 2048)
    n_arr = (ctypes.c_int32 * 3)(*ns)
    a_arr = (ctypes.c_double * 3)(1.5, 1.5, 1.5)
    h_arr = (ctypes.c_double * 3)(*W.mesh_widths(ns))
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = L.sfac_solve_noalloc(3, n_arr, a_arr, 0.1, 0.01, h_arr, sfac.FP64, ctypes.c_void_p(one.data_ptr()), 1,
                              None, None, None, None)
    assert st == sfac.EUNSUPPORTED and b"workspace" in L.sfac_last_error()
    with pytest.raises(sfac.SfacError) as err:
        sfac.solve_noalloc(u, inst.ns, inst.alphas, inst.eps, inst.tau, inst.hs, -1)
    assert err.value.status == sfac.EINVAL
