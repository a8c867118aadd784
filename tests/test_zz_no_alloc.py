"""The allocation-free solve (sem_pcg_solve_noalloc) against sem_pcg_solve:
the same kernels on a workspace in the library's static device scratch, so
solutions and reports must be identical bit for bit.  Two calls in a row,
the second on a smaller mesh (the scratch keeps the first call's contents),
plus the size limit, checked before any device work."""
import numpy as np
import pytest

from paper_2405_05640_amd import sem
from paper_2405_05640_amd import workloads as wl
from tests.gpu_util import dev, host, pair

pytestmark = pytest.mark.gpu


def _solve_both(spec, form, prepare=0, **kw):
    import torch
    om, gm = pair(spec, prepare=prepare)
    rng = np.random.default_rng(7)
    b = dev(om.rhs(rng.standard_normal(om.shape)))
    x_ref = torch.zeros_like(b)
    r_ref = gm.pcg_solve(b, x_ref, form=form, **kw)
    x = torch.full_like(b, float("nan"))     # the solve must not read x
    r = gm.pcg_solve_noalloc(b, x, form=form, **kw)
    torch.cuda.synchronize()
    assert torch.equal(x, x_ref)
    for f in ("status", "iterations", "outer_iterations", "restarts", "rel_res", "true_rel_res"):
        assert getattr(r, f) == getattr(r_ref, f), f
    rh = host(b) - om.apply_S(host(x), kw.get("h1", 1.0), kw.get("h2", 0.0))
    assert np.sqrt(om.dot(rh, rh) / om.dot(host(b), host(b))) <= 1.05e-10
    return r


@pytest.mark.parametrize("form,prepare,kw", [
    (sem.FORM_JACOBI_PCG, 0, {"h2": 0.1}),
    (sem.FORM_RELIABLE_FP32, sem.SEM_PREP_F32, {"inner_tol": 0.1}),
    (sem.FORM_GMRES_HSMG, sem.SEM_PREP_HSMG, {"restart": 10}),
    (sem.FORM_PCG_HSMG, sem.SEM_PREP_HSMG, {"h2": 0.1}),
], ids=["fp64_pcg", "reliable_fp32", "gmres_hsmg", "pcg_hsmg"])
def test_noalloc_matches_workspace_solve_twice(form, prepare, kw):
    # first a larger mesh, then a smaller one on the same scratch
    r1 = _solve_both(wl.random_deformed_box(6, 5, 4, 7, seed=3, amp=0.1), form, prepare, **kw)
    r2 = _solve_both(wl.random_deformed_box(3, 2, 2, 5, seed=4, amp=0.1), form, prepare, **kw)
    print("noalloc form %d: %d then %d iterations" % (form, r1.iterations, r2.iterations))


def test_noalloc_rejects_meshes_beyond_the_scratch():
    import torch
    gm = sem.Mesh.from_spec(wl.deformed_cube(16, 7))      # 2.1 M local points: about 70 MiB of workspace
    opts = gm.solve_opts()
    assert gm.workspace_bytes(opts) > sem.NOALLOC_SCRATCH_BYTES
    b = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(sem.SemError) as exc:
        gm.pcg_solve_noalloc(b, x)
    assert exc.value.status == sem.SEM_ERR_INVALID_ARG
    assert "static scratch" in str(exc.value)
