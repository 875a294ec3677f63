"""The serving loop (srv_* entry points): requests of different families,
sizes and ranks, admitted by slots and by the free space of a device pool,
overlapping on the device.  In deterministic mode every result is bitwise
the same alone, in the mix, and from a reduced-model handle driven directly."""
import numpy as np
import pytest

from workloads import workload
from workloads.ensembles import draw_parameters, philox_uniforms

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def _b():
    import torch
    from paper_2201_05555_amd import binding
    assert torch.cuda.is_available()
    return binding, torch


def _requests(binding):
    """Six requests: both families, p from 3 to 70, N from 6000 to 30000,
    ranks 8 to 16, Galerkin and DEIM, 12 to 30 steps."""
    specs = [("landau_tiny", 3, 6000, 64, 8, "galerkin", 12),
             ("twostream_deim", 17, 20000, 128, 10, "deim", 20),
             ("twostream_deim", 40, 12000, 64, 16, "galerkin", 15),
             ("landau_tiny", 24, 30000, 64, 10, "galerkin", 18),
             ("twostream_deim", 70, 8000, 96, 12, "deim", 30),
             ("twostream_deim", 9, 25000, 128, 8, "galerkin", 25)]
    out = []
    for j, (name, p, N, Nx, two_n, proj, steps) in enumerate(specs):
        w = workload(name, p=p, N=N, Nx=Nx)
        params = draw_parameters(w, seed=1000 * w["number"] + 11 + j)
        ux, uv = philox_uniforms(7000 + j, N)
        cfg = binding.make_config(N, p, Nx, two_n, two_n_max=two_n + 4, dt=w["dt"],
                                  projection=proj, deim_window=3, fp_tol=1e-10,
                                  rank_auto=True, rank_tol_up=1e-2, deterministic=True)
        rows = np.array([0, N // 3, N - 1], dtype=np.int32)
        out.append(dict(cfg=cfg, family=w["family"], params=params, ux=ux, uv=uv,
                        steps=steps, rows=rows))
    return out


def _run(binding, reqs, slots, pool_bytes):
    srv = binding.Server(slots, pool_bytes)
    ids = [srv.submit(q["cfg"], q["family"], q["params"], q["ux"], q["uv"], q["steps"],
                      q["rows"]) for q in reqs]
    srv.drain()
    res = [srv.result(i) for i in ids]
    infos = [srv.info(i) for i in ids]
    srv.close()
    return res, infos


def test_serving_alone_equals_mix():
    binding, torch = _b()
    reqs = _requests(binding)
    _say("serving alone vs mix", len(reqs))
    need = [binding.lib().srv_request_bytes(q["cfg"], len(q["rows"])) for q in reqs]
    alone = []
    for q in reqs:
        r, inf = _run(binding, [q], 1, 2 * max(need))
        assert inf[0]["status"] == 0 and inf[0]["steps_done"] == q["steps"]
        alone.append(r[0])
    mix, infos = _run(binding, reqs, 4, sum(need) + (1 << 20))
    # the requests did run side by side
    ivs = sorted((i["t_start"], i["t_finish"]) for i in infos)
    overlap = any(ivs[k + 1][0] < ivs[k][1] for k in range(len(ivs) - 1))
    print(f"  requests overlapped on the device: {overlap}", flush=True)
    for a, m in zip(alone, mix):
        for x, y in zip(a, m):
            assert np.array_equal(x, y)


def test_serving_matches_a_direct_handle():
    """A request's energies and rows equal those of a reduced-model handle
    initialised from the same inputs and stepped the same number of times."""
    binding, torch = _b()
    q = _requests(binding)[1]
    _say("serving vs direct handle")
    need = binding.lib().srv_request_bytes(q["cfg"], len(q["rows"]))
    res, inf = _run(binding, [q], 1, need + (1 << 20))
    E, H, X, V = res[0]
    r = binding.Rom(q["cfg"], None, None, None, family=q["family"], params=q["params"],
                    ux=q["ux"], uv=q["uv"])
    r.step(q["steps"])
    E2, H2 = r.diagnostics()
    X2, V2 = r.reconstruct_rows(q["rows"])
    assert np.array_equal(E, E2.cpu().numpy())
    assert np.array_equal(H, H2.cpu().numpy())
    assert np.array_equal(X, X2.cpu().numpy()) and np.array_equal(V, V2.cpu().numpy())


def test_serving_admission_by_pool_space():
    """With room in the pool for two requests at a time (and four slots), no
    more than two run at once, and all finish."""
    binding, torch = _b()
    reqs = [q for q in _requests(binding)]
    for j, q in enumerate(reqs):   # same shape for a clean capacity bound
        q["cfg"].N, q["cfg"].p, q["cfg"].Nx = 12000, 16, 64
        q["ux"], q["uv"] = philox_uniforms(9000 + j, 12000)
        q["params"] = {k: v[:16] if len(v) >= 16 else np.resize(v, 16)
                       for k, v in q["params"].items()}
        q["rows"] = np.array([0, 5], dtype=np.int32)
        q["cfg"].two_n, q["cfg"].two_n_max = 8, 8
        q["cfg"].projection = binding.GALERKIN
    _say("serving admission by pool space")
    need = max(binding.lib().srv_request_bytes(q["cfg"], 2) for q in reqs)
    res, infos = _run(binding, reqs, 4, 2 * need + 4096)
    assert all(i["status"] == 0 for i in infos)
    ev = sorted([(i["t_start"], 1) for i in infos] + [(i["t_finish"], -1) for i in infos])
    cur = peak = 0
    for _, d in ev:
        cur += d
        peak = max(peak, cur)
    print(f"  peak concurrent requests {peak}", flush=True)
    assert peak <= 2
