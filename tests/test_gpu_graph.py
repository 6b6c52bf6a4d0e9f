"""The matvec + SMW apply step captured as a HIP graph: every replay, with
eager work and synchronisations in between, equals the eager result
bitwise (the kernels are deterministic and record no memset nodes)."""
import pytest
import torch

from gpu_util import DEV, log, to_dev, vec
from paper_2403_09198_amd import gen, r1s

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,ny,L,nrhs", [(32, 16, 61, 1), (8, 8, 200, 2)])
def test_graph_replays_match_eager(nx, ny, L, nrhs):
    log(f"graph replay nx={nx} ny={ny} L={L} nrhs={nrhs}")
    p = gen.make_problem(nx, ny, L, seed=3)
    A = r1s.R1Matrix(nx, ny, L, to_dev(p), keep_f32=True)
    M = r1s.SMWPreconditioner(A, keep_f32=True, with_trans=True)
    x = vec(gen.make_vector(nx, ny, L, nrhs=nrhs, seed=1))
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    zt = torch.empty_like(x)

    def step():
        A.matvec(x, out=y)
        M.apply(y, out=z)
        M.apply(y, out=zt, trans=True, precision="f32")

    step()
    torch.cuda.synchronize()
    ref = (y.clone(), z.clone(), zt.clone())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for i in range(4):
        y.zero_(); z.zero_(); zt.zero_()
        junk = A.matvec(vec(gen.make_vector(nx, ny, L, nrhs=nrhs, seed=10 + i)))  # eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref[0]) and torch.equal(z, ref[1]) and torch.equal(zt, ref[2]), i
        del junk
