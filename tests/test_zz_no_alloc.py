"""GPU test of the allocation-free energy entry point: through the C ABI it
gives the energy of ccfmm_plan_energy_device (same kernels, same summation
order, so bitwise equal) and the oracle's energy to 1e-12, on two calls in a
row, the second with fewer dipoles and configurations than the first."""
import numpy as np
import pytest

from paper_0810_0233_amd import ccfmm, inputs

pytestmark = pytest.mark.gpu


def test_noalloc_energy_matches_plan_energy(ref):
    import torch

    st = torch.cuda.current_stream().cuda_stream
    for (nx, ny, nz), nb, seed in (((12, 12, 12), 3, 61), ((7, 8, 9), 2, 62)):
        pos, box = inputs.lattice(nx, ny, nz)
        n = pos.shape[0]
        print("case lattice %dx%dx%d n=%d nbatch=%d" % (nx, ny, nz, n, nb), flush=True)
        m = np.stack([inputs.random_moments(n, seed + b) for b in range(nb)])
        prm = ccfmm.params(order=4, theta=0.5, leaf_target=8, box=box, max_batch=nb)
        pl = ccfmm.Plan.create(pos, prm)
        H = pl.eval(m)
        dm = torch.from_numpy(np.ascontiguousarray(m)).to("cuda:0")
        dH = torch.from_numpy(np.ascontiguousarray(H)).to("cuda:0")
        E_plan = torch.full((nb,), float("nan"), dtype=torch.float64, device="cuda:0")
        E_na = torch.full((nb,), float("nan"), dtype=torch.float64, device="cuda:0")
        pl.energy_device(nb, dm.data_ptr(), dH.data_ptr(), E_plan.data_ptr(), st)
        ccfmm.energy_device_noalloc(n, nb, dm.data_ptr(), dH.data_ptr(), E_na.data_ptr(), st)
        torch.cuda.synchronize()
        e_plan, e_na = E_plan.cpu().numpy(), E_na.cpu().numpy()
        assert np.array_equal(e_na, e_plan), (e_na, e_plan)
        e_ref = np.array([ref.energy(m[b], H[b]) for b in range(nb)])
        assert np.all(np.abs(e_na - e_ref) <= 1e-12 * np.abs(e_ref)), (e_na, e_ref)
        pl.destroy()
