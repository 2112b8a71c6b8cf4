"""The inference entry point that allocates nothing (nfm_mlp_infer_bf16_noalloc) against the one
that uses the network's workspace (nfm_mlp_infer_bf16), through the C ABI: bit for bit on two
calls in a row, the second with fewer rows (what the first left in the static scratch must not
show), a batch above the network's batch_max, and the size limit refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_08560_amd import nfm as m
    m.lib()
    return m


def _reference(mlp, x):
    import torch
    out = torch.empty((x.shape[0], 256), dtype=torch.float32, device=x.device)
    for s in range(0, x.shape[0], mlp.batch_max):
        mlp.infer_bf16(x[s:s + mlp.batch_max].contiguous(), out=out[s:s + mlp.batch_max])
    return out


def test_noalloc_inference_matches_workspace_inference(nfm):
    import torch
    rng = np.random.default_rng(5)
    mlp = nfm.Mlp(batch_max=128)
    mlp.init(99)
    p, _ = mlp.get_params()
    p = p + rng.normal(0, 0.05, p.shape).astype(np.float32)          # nonzero biases
    norm = np.stack([rng.normal(0, 1, 81), rng.uniform(0.5, 2, 81)]).astype(np.float32)
    mlp.set_params(p, norm)
    mlp.to_bf16()
    for rows in (1000, 37):                                             # second call smaller
        print(f"no-alloc inference: {rows} rows", flush=True)
        x = torch.tensor(rng.normal(0, 1.5, (rows, 81)).astype(np.float32), device="cuda")
        y = torch.full((rows, 256), float("nan"), dtype=torch.float32, device="cuda")
        mlp.infer_bf16_noalloc(x, y)
        ref = _reference(mlp, x)
        torch.cuda.synchronize()
        yc, rc = y.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(yc).all()
        assert np.array_equal(yc.view(np.uint32), rc.view(np.uint32)), rows
    lib = nfm.lib()
    x = torch.zeros((1025, 81), dtype=torch.float32, device="cuda")
    y = torch.zeros((1025, 256), dtype=torch.float32, device="cuda")
    assert lib.nfm_mlp_infer_bf16_noalloc(mlp.ctx, x.data_ptr(), 1025, y.data_ptr()) == nfm.NFM_ERANGE
    assert "1024" in lib.nfm_mlp_last_error(mlp.ctx).decode()
    assert lib.nfm_mlp_infer_bf16_noalloc(mlp.ctx, x.data_ptr(), 0, y.data_ptr()) == nfm.NFM_EINVAL
    mlp.close()
