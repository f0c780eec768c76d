"""The allocation-free projected operator (for callers that cannot allocate
device memory) against bgcr_apply_projected with a caller-owned workspace:
same kernels, so the results must agree to the bit; two calls in a row, the
second on a smaller input, and the size limit of the library's workspace."""
import numpy as np
import pytest

import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(bg, dev, n, p, kdim, seed):
    A = problems.banded(n, 9, seed=seed)
    rng = np.random.default_rng(seed + 1)
    C, _ = np.linalg.qr(rng.uniform(-1, 1, (n, kdim)))
    kc = -(-kdim // p)
    Cb = np.zeros((kc, n, p))
    for c in range(kdim):
        Cb[c // p, :, c % p] = C[:, c]
    V = rng.uniform(-1, 1, (n, p))
    return (bg.DeviceCSR.from_scipy(A, dev), torch.from_numpy(Cb).to(dev), torch.from_numpy(V).to(dev), kc)


@pytest.mark.parametrize("p", [1, 2, 8, 16])
@pytest.mark.parametrize("variant", [0, 1])
def test_noalloc_matches_workspace_entry_point(p, variant):
    import paper_1604_01713_amd as bg
    assert torch.cuda.is_available(), "GPU test without a GPU"
    dev = torch.device("cuda:0")
    # the second call is smaller (n and dim C): whatever the first left in
    # the library's workspace must not leak into it
    for n, kdim, seed in ((20011, 40, 5), (3001, 10, 9)):
        Ad, Cd, Vd, kc = _case(bg, dev, n, p, kdim, seed)
        W_ref = torch.full_like(Vd, 3.0)
        work = torch.empty(bg.bgcr_apply_projected_work_bytes(n, p, kc), dtype=torch.uint8, device=dev)
        bg.bgcr_apply_projected(Ad, Cd, Vd, W_ref, variant, work)
        W_na = torch.full_like(Vd, -5.0)
        bg.bgcr_apply_projected_noalloc(Ad, Cd, Vd, W_na, variant)
        torch.cuda.synchronize()
        diff = float((W_na - W_ref).abs().max())
        print(f"noalloc p={p} variant={variant} n={n} dim C={kdim}: max |diff| {diff:.1e}", flush=True)
        assert torch.equal(W_na, W_ref)
        assert float(W_ref.abs().max()) > 0.0


def test_noalloc_rejects_sizes_beyond_its_workspace():
    import paper_1604_01713_amd as bg
    assert torch.cuda.is_available(), "GPU test without a GPU"
    dev = torch.device("cuda:0")
    n, p = 1000, 16
    kc_max = (bg.BGCR_NOALLOC_SCRATCH_BYTES // 8 - 512 * 17 * p * p) // (p * p)
    assert bg.bgcr_apply_projected_work_bytes(n, p, kc_max) <= bg.BGCR_NOALLOC_SCRATCH_BYTES
    assert bg.bgcr_apply_projected_work_bytes(n, p, kc_max + 1) > bg.BGCR_NOALLOC_SCRATCH_BYTES
    Ad, _, Vd, _ = _case(bg, dev, n, p, 16, 3)
    C = torch.zeros((kc_max + 1, 1, p), dtype=torch.float64, device=dev)  # shape only: rejected before any launch
    W = torch.zeros_like(Vd)
    with pytest.raises(bg.BgcrError) as e:
        bg.bgcr_apply_projected_noalloc(Ad, C, Vd, W, 0)
    assert e.value.code == bg.BGCR_ERR_INVALID
