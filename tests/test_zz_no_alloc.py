"""GPU check of icp_point_to_plane_noalloc (the entry point for callers that
cannot allocate: it runs on the library's static device scratch) against
icp_point_to_plane with a caller workspace, through the C ABI.  Two calls in
a row on one GPU, the second with a smaller pair, each equal to the
workspace form bit for bit (same kernels, same inputs)."""
import numpy as np
import pytest

from gen import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_00399_amd import pcgpu
    return pcgpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pair(oracle_mod, cfg, size):
    w = make_workload(cfg, size=size)
    nrm, _, _ = oracle_mod.normals(w.target, w.k, (0.0, 0.0, 0.0))
    return w, nrm.astype(np.float32)


def test_noalloc_equals_workspace_form_twice(gpu, oracle_mod):
    import torch
    # first a 307,200-point room pair (near the scratch limit), then a
    # 2,000-point sphere+plane pair: the second call must not see the first
    # call's scratch contents
    for cfg, size in ((1, "full"), (0, "small")):
        w, nrm = _pair(oracle_mod, cfg, size)
        print(f"noalloc {w.name} n={w.n} iters={w.iters}", flush=True)
        S, T, N = _dev(w.source), _dev(w.target), _dev(nrm)
        T0 = torch.eye(4, dtype=torch.float64, device="cuda")
        out_T = torch.full((4, 4), float("nan"), dtype=torch.float64, device="cuda")
        out_st = torch.zeros(24, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        gpu.icp_point_to_plane_noalloc(S, T, N, out_T, out_st, T0, w.d_max, w.iters)
        Tr, sr = gpu.icp_point_to_plane(S, T, N, T0, w.d_max, w.iters)
        torch.cuda.synchronize()
        s_no = gpu.decode_stats(out_st)
        assert torch.equal(out_T, Tr), (out_T.cpu().numpy(), Tr.cpu().numpy())
        assert s_no == sr, (s_no, sr)
        ro = oracle_mod.icp(w.source, w.target, nrm, None, float(np.float32(w.d_max)), w.iters)
        Tn = out_T.cpu().numpy()
        assert np.abs(Tn - ro["T"]).max() < 1e-6 and s_no["inliers"] == ro["inliers"]


def test_noalloc_rejects_requests_beyond_its_scratch(gpu):
    import torch
    n = 400_000
    x = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    out_T = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    out_st = torch.zeros(24, dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu.PcgpuError) as e:
        gpu.icp_point_to_plane_noalloc(x, x, x, out_T, out_st, None, 0.05, 30)
    assert e.value.status == gpu.PC_EWORKSPACE
