"""Graph capture of the single-pair path: icp_point_to_plane_with_normals
launches kernels only (no memset, no host copy), so with its workspace and
outputs preallocated it can be captured once and replayed.  Every replay,
with eager work and synchronisation between replays, must equal the eager
result bit for bit."""
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


@pytest.mark.parametrize("cfg,size", [(0, "full"), (1, "small")])
def test_graph_replays_equal_eager(gpu, cfg, size):
    import torch
    w = make_workload(cfg, size=size)
    print(f"graph {w.name} n={w.n}", flush=True)
    dev = torch.device("cuda:0")
    src = torch.from_numpy(w.source).to(dev)
    tgt = torch.from_numpy(w.target).to(dev)
    ws = torch.empty(gpu.lib.icp_point_to_plane_with_normals_workspace_size(w.n, w.n, w.iters), dtype=torch.uint8,
                     device=dev)
    T = torch.empty((4, 4), dtype=torch.float64, device=dev)
    st = torch.zeros(24, dtype=torch.uint8, device=dev)
    nrm = torch.empty((w.n, 3), dtype=torch.float32, device=dev)

    def step():
        gpu.icp_point_to_plane_with_normals(src, tgt, w.k, (0.0, 0.0, 0.0), None, w.d_max, w.iters, workspace=ws,
                                            out_T=T, out_stats=st, read_stats=False, out_normals=nrm)

    step()
    torch.cuda.synchronize()
    ref = (T.clone(), st.clone(), nrm.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):          # warm-up on the side stream, as capture requires
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    other = make_workload(0, size="small")
    osrc, otgt = torch.from_numpy(other.source).to(dev), torch.from_numpy(other.target).to(dev)
    for rep in range(4):
        T.zero_()
        st.zero_()
        nrm.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(T, ref[0]) and torch.equal(st, ref[1]) and torch.equal(nrm, ref[2]), rep
        # eager work of the program between replays
        gpu.icp_point_to_plane_with_normals(osrc, otgt, other.k, max_corr_dist=other.d_max, max_iters=other.iters)
        torch.cuda.synchronize()


def test_batched_graph_replays_equal_eager(gpu):
    """The batched call passes its host offsets and per-pair parameters as
    kernel arguments, so it too launches kernels only and can be captured;
    every replay must equal the eager result bit for bit."""
    import torch
    from gen import batch_workload
    b = batch_workload(3, "small")
    print(f"batched graph {b.name} pairs={b.n_pairs} n={b.n}", flush=True)
    dev = torch.device("cuda:0")
    off = b.offsets
    m = b.n_pairs
    k, dm, it = b.param("k").astype(np.int32), b.param("d_max").astype(np.float32), b.param("iters").astype(np.int32)
    src = torch.from_numpy(b.source).to(dev)
    tgt = torch.from_numpy(b.target).to(dev)
    ws = torch.empty(gpu.lib.icp_point_to_plane_with_normals_batched_workspace_size(m, off.ctypes.data,
                                                                                    off.ctypes.data, int(it.max())),
                     dtype=torch.uint8, device=dev)
    T = torch.empty((m, 4, 4), dtype=torch.float64, device=dev)
    st = torch.zeros(24 * m, dtype=torch.uint8, device=dev)
    nrm = torch.empty((b.target.shape[0], 3), dtype=torch.float32, device=dev)

    def step():
        gpu.icp_point_to_plane_with_normals_batched(src, off, tgt, off, k, (0.0, 0.0, 0.0), None, dm, it,
                                                    workspace=ws, out_T=T, out_stats=st, read_stats=False,
                                                    out_normals=nrm)

    step()
    torch.cuda.synchronize()
    ref = (T.clone(), st.clone(), nrm.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        T.zero_()
        st.zero_()
        nrm.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(T, ref[0]) and torch.equal(st, ref[1]) and torch.equal(nrm, ref[2]), rep
        # eager work between replays: the same call on other arrays
        gpu.icp_point_to_plane_with_normals_batched(tgt, off, src, off, k, (0.0, 0.0, 0.0), None, dm, it)
        torch.cuda.synchronize()
