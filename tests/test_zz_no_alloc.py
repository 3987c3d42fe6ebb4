"""tmm_rt_grad_noalloc (static scratch, no allocation) against tmm_rt_grad:
the same gradients, bit for bit, on two calls in a row -- the 1024 x 60-layer
adjoint batch (capped persistent grid, several launches inside the scratch),
then a smaller batch that leaves the first call's contents in the scratch --
and a batch too large for the scratch rejected with TMM_ERR_WORKSPACE."""
import numpy as np
import pytest

from paper_2111_13667_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def both(w, gR, gT=None):
    from paper_2111_13667_amd import tmm
    args = (dev(w.d, torch.float64), dev(w.nk, torch.complex128), dev(w.wl, torch.float64),
            dev(w.sin_t, torch.float64), dev(w.cos_t, torch.float64))
    mat = None if w.mat is None else dev(w.mat, torch.int32)
    out = []
    for fn in (tmm.tmm_rt_grad, tmm.tmm_rt_grad_noalloc):
        gd = torch.full((w.B, w.L), 7.0, dtype=torch.float64, device="cuda")
        gn = torch.full((w.B, w.L), 7.0, dtype=torch.complex128, device="cuda")
        R = torch.empty((w.B, 2, w.theta.size, w.wl.size), dtype=torch.float64, device="cuda")
        fn(*args, mat=mat, dl_dR=dev(gR, torch.float64), dl_dT=None if gT is None else dev(gT, torch.float64),
           grad_d=gd, grad_n=gn, R=R)
        torch.cuda.synchronize()
        out.append((gd.cpu().numpy(), gn.cpu().numpy(), R.cpu().numpy()))
    return out


def test_noalloc_matches_workspace_entry_point_on_two_calls():
    from paper_2111_13667_amd import tmm
    assert tmm.library().tmm_rt_grad_noalloc_scratch_bytes() == 192 << 20
    # call 1: the adjoint batch; its preferred workspace (checkpoints of the full
    # persistent grid + partial sums) is larger than the scratch
    w = workloads.adjoint_batch()
    print("noalloc call 1: adjoint batch", w.B, "x", w.L, "x", w.wl.size, "x", w.theta.size, flush=True)
    rng = np.random.default_rng(7)
    gR = rng.normal(size=(w.B, 2, w.theta.size, w.wl.size)) / 1e6
    (gd0, gn0, R0), (gd1, gn1, R1) = both(w, gR)
    assert np.isfinite(gd0).all() and np.isfinite(gn0).all()
    assert np.array_equal(gd0, gd1) and np.array_equal(gn0, gn1) and np.array_equal(R0, R1)
    # call 2: a smaller batch with per-layer rows (the division-free adjoint) and dl/dT
    w2 = workloads.random_stacks(8, B=9, L=13, n_wl=70, n_theta=3)
    print("noalloc call 2: random stacks", w2.B, "x", w2.L, "x", w2.wl.size, "x", w2.theta.size, flush=True)
    shape = (w2.B, 2, w2.theta.size, w2.wl.size)
    (gd0, gn0, R0), (gd1, gn1, R1) = both(w2, rng.normal(size=shape), rng.normal(size=shape))
    assert np.isfinite(gd0).all()
    assert np.array_equal(gd0, gd1) and np.array_equal(gn0, gn1) and np.array_equal(R0, R1)


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    from paper_2111_13667_amd import tmm
    # 1000 layers over 4096 wavelengths x 91 angles: one stack's partial sums
    # alone (140 MB) leave no room beside the checkpoints
    w = workloads.random_stacks(5, B=4, L=1000, n_wl=4096, n_theta=91)
    args = (dev(w.d, torch.float64), dev(w.nk, torch.complex128), dev(w.wl, torch.float64),
            dev(w.sin_t, torch.float64), dev(w.cos_t, torch.float64))
    gR = torch.zeros((w.B, 2, w.theta.size, w.wl.size), dtype=torch.float64, device="cuda")
    gd = torch.full((w.B, w.L), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(tmm.TmmError) as e:
        tmm.tmm_rt_grad_noalloc(*args, dl_dR=gR, grad_d=gd)
    assert e.value.status == tmm.TMM_ERR_WORKSPACE
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert (gd == 7.0).all()
