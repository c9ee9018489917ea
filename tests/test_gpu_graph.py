"""GMRES with its preconditioner replayed as a captured HIP graph.

After the first application, the sweep launches of one preconditioner
application are captured once and the graph is replayed at every later Arnoldi
step, with the Krylov kernels, host read-backs and synchronizations of the
method in between.  Every replay feeds the next Krylov vector, so the final
iterate depends on each of them: it must equal, bit for bit, the result of the
same GMRES with direct launches (lrx_tune solve_graph = 0), for one system and
for a batch, over several calls in a row on the same handles (graphs are
captured per call).  Runs on a non-blocking torch stream (the null stream is
never captured).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from parity_util import TOL, grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1510_07363_amd import lorax
    return lorax, torch


def _run(lx, torch, Fs, bs, nrhs, graph):
    base = lx.tune_get()
    lx.tune_set(solve_graph=1 if graph else 0)
    try:
        xs = [torch.zeros_like(b) for b in bs]
        if len(Fs) == 1:
            its, rr, st = Fs[0].gmres_dev(bs[0].data_ptr(), xs[0].data_ptr(), nrhs, tol=TOL, restart=30, maxit=200)
        else:
            its, rr, st = lx.gmres_batch_dev(Fs, nrhs, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs],
                                             tol=TOL, restart=30, maxit=200)
        torch.cuda.synchronize()
        return xs, np.asarray(its).copy(), st
    finally:
        lx.tune_set(**base)


def test_graph_replays_equal_direct_launches(env):
    lx, torch = env
    stream = torch.cuda.Stream()
    ins = [grid("varcoef2d", 64, 32, 1), grid("lognormal3d", 12, 32, 2)]
    nrhs = 3
    with torch.cuda.stream(stream):
        sptr = stream.cuda_stream
        Fs = [lx.Factor(*csr, perm, lp, depth, 1e-2, stream=sptr, precision=prec)
              for (csr, n, perm, lp, depth, _), prec in zip(ins, ("fp64", "mixed"))]
        bs = [torch.from_numpy(rng.uniform(-1, 1, (nrhs, n))).to("cuda:0") for (_, n, _, _, _, rng) in ins]
        torch.cuda.synchronize()
        for rep in range(2):                                    # calls in a row on the same handles
            for sel in ([0], [1], [0, 1]):
                F_sel, b_sel = [Fs[i] for i in sel], [bs[i] for i in sel]
                x_g, it_g, st_g = _run(lx, torch, F_sel, b_sel, nrhs, True)
                x_d, it_d, st_d = _run(lx, torch, F_sel, b_sel, nrhs, False)
                assert st_g == st_d == lx.LRX_OK
                assert np.array_equal(it_g, it_d) and it_g.max() >= 3     # several replays per cycle
                for xg, xd in zip(x_g, x_d):
                    assert torch.equal(xg, xd), float((xg - xd).abs().max())
                for i, xg in zip(sel, x_g):
                    csr, n, perm, lp, depth, _ = ins[i]
                    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
                    X, B = xg.cpu().numpy().T, bs[i].cpu().numpy().T
                    assert (np.linalg.norm(A @ X - B, axis=0) / np.linalg.norm(B, axis=0) <= TOL).all()


def test_capture_beside_factorizations_in_another_thread(env):
    """A serving process factors in one thread while another solves: the
    factorization's synchronous host copies (null stream) must wait for a graph
    capture in progress instead of failing.  Factorizations (host values, so
    each one copies them) run back to back in a worker thread while this thread
    runs GMRES calls that each capture their preconditioner; every call
    succeeds and reaches the true residual."""
    import threading
    lx, torch = env
    csr, n, perm, lp, depth, rng = grid("varcoef2d", 64, 32, 3)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
    fs = torch.cuda.Stream()
    errors, count = [], [0]
    stop = threading.Event()

    def factor_loop():
        try:
            torch.cuda.set_device(0)
            while not stop.is_set():
                F = lx.Factor(*csr, perm, lp, depth, 1e-3, stream=fs.cuda_stream, precision="mixed")
                F.free()
                count[0] += 1
        except Exception as e:                      # reported by the main thread
            errors.append(e)

    ss = torch.cuda.Stream()
    base = lx.tune_get()
    lx.tune_set(solve_graph=1)
    try:
        with torch.cuda.stream(ss):
            F = lx.Factor(*csr, perm, lp, depth, 1e-3, stream=ss.cuda_stream, precision="mixed")
            b = torch.from_numpy(rng.uniform(-1, 1, (2, n))).to("cuda:0")
            torch.cuda.synchronize()
            th = threading.Thread(target=factor_loop)
            th.start()
            try:
                for _ in range(30):
                    x = torch.zeros_like(b)
                    its, rr, st = F.gmres_dev(b.data_ptr(), x.data_ptr(), 2, tol=TOL, restart=30, maxit=200)
                    ss.synchronize()
                    assert st == lx.LRX_OK and min(its) >= 3
                    X, B = x.cpu().numpy().T, b.cpu().numpy().T
                    assert (np.linalg.norm(A @ X - B, axis=0) / np.linalg.norm(B, axis=0) <= TOL).all()
            finally:
                stop.set()
                th.join()
    finally:
        lx.tune_set(**base)
    print(f"{count[0]} factorizations beside 30 captured GMRES calls")
    assert not errors, errors[0]
    assert count[0] >= 1
