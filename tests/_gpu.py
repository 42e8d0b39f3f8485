"""Helpers for the GPU tests: run the library through its C ABI (via the
ctypes binding) on device buffers and bring the results back as numpy."""
import numpy as np
import torch

from paper_2308_01037_amd import mcmf as M

FN = {"exp": M.MCMF_FN_EXP, "resolvent": M.MCMF_FN_RESOLVENT}


def fn_struct(fn, scale):
    if isinstance(fn, str):
        return M.make_fn(FN[fn], scale)
    return M.make_fn(M.MCMF_FN_COEFFS, scale, coeffs=np.asarray(fn, dtype=np.float64))


def oracle_fn(fn):
    import oracle
    if isinstance(fn, str):
        return {"exp": oracle.FN_EXP, "resolvent": oracle.FN_RESOLVENT}[fn]
    return np.asarray(fn, dtype=np.float64)


def default_sampler(csr):
    """The oracle's sampler mode for the library's default layout: weighted
    rows walk by the alias method, unweighted rows are not affected."""
    return "alias" if getattr(csr, "val", None) is not None else "cdf"


def graph(csr, flags=M.MCMF_SYMMETRIC):
    return M.Graph.from_csr(csr, flags=flags)


def gpu_action(g, fn, v, N, K, scale=1.0, seed=0, request=0, cutoff=0.0, want_q=False,
               want_digest=False, stats=False, host=False):
    n = g.info["n"]
    dev = "cpu" if host else "cuda"
    vt = torch.as_tensor(np.asarray(v, dtype=np.float64), device=dev).contiguous()
    out = torch.empty(n, dtype=torch.float64, device=dev)
    q = torch.zeros(n, dtype=torch.float64, device=dev) if want_q else None
    dig = torch.zeros(n, dtype=torch.int64, device=dev) if want_digest else None
    st = M.mcmf_stats() if stats else None
    stream = None if host else torch.cuda.current_stream().cuda_stream
    opts = M.make_opts(seed=seed, request_id=request, weight_cutoff=cutoff, stream=stream,
                       path_digest=dig, q_out=q)
    M.mcmf_action(g.handle, fn_struct(fn, scale), vt, N, K, opts, out, st)
    if not host:
        torch.cuda.synchronize()
    res = {"y": out.cpu().numpy()}
    if want_q:
        res["q"] = q.cpu().numpy()
    if want_digest:
        res["digest"] = dig.cpu().numpy().view(np.uint64)
    if stats:
        res["stats"] = st.as_dict()
    return res


def gpu_diag(g, fn, N, K, scale=1.0, seed=0, request=0, cutoff=0.0, rows=None,
             want_digest=False, stats=False, host=False):
    n = g.info["n"]
    dev = "cpu" if host else "cuda"
    rt = None if rows is None else torch.as_tensor(np.asarray(rows, dtype=np.int32), device=dev)
    count = n if rows is None else len(rows)
    out = torch.empty(max(count, 1), dtype=torch.float64, device=dev)
    dig = torch.zeros(n, dtype=torch.int64, device=dev) if want_digest else None
    st = M.mcmf_stats() if stats else None
    stream = None if host else torch.cuda.current_stream().cuda_stream
    opts = M.make_opts(seed=seed, request_id=request, weight_cutoff=cutoff, stream=stream,
                       path_digest=dig)
    M.mcmf_diag(g.handle, fn_struct(fn, scale), rt, 0 if rows is None else len(rows), N, K, opts,
                out, st)
    if not host:
        torch.cuda.synchronize()
    res = {"d": out.cpu().numpy()[:count]}
    if want_digest:
        res["digest"] = dig.cpu().numpy().view(np.uint64)
    if stats:
        res["stats"] = st.as_dict()
    return res


def assert_close(got, want, rtol=1e-10, atol=0.0, what=""):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    err = np.abs(got - want)
    bound = rtol * np.abs(want) + atol
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (f"{what}: {bad.size} entries off; first {bad[:5]}, got {got[bad[:5]]}, "
                           f"want {want[bad[:5]]}")


def assert_mc_part_close(got, want, h, rtol=1e-10, what=""):
    """Compare the Monte Carlo parts x - h element-wise; the subtraction
    itself may lose up to a few ulps of |x|."""
    got, want, h = map(np.asarray, (got, want, h))
    u_got, u_want = got - h, want - h
    atol = 8 * np.finfo(np.float64).eps * np.abs(want)
    err = np.abs(u_got - u_want)
    bad = np.nonzero(err > rtol * np.abs(u_want) + atol)[0]
    assert bad.size == 0, (f"{what}: MC part off at {bad[:5]}: {u_got[bad[:5]]} vs {u_want[bad[:5]]}")
