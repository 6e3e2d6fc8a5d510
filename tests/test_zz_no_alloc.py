"""The allocation-free growth-map entry point (qs_growth_map_noalloc) against the allocating
one (qs_growth_map): answers (baseline + network) bit for bit equal to its SURROGATE mode and
routing flags equal to the queries its AUTO mode sends to the solver, over two calls in a row
on one device (the second smaller, so it reuses the library's scratch array), plus the size
limit."""
import ctypes
import math

import numpy as np
import pytest

from oracle import growth as Gr
from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _net(qs, seed):
    rng = np.random.default_rng(seed)
    P = [(np.float32(W).astype(np.float64), np.float32(b).astype(np.float64)) for W, b in M.init_params(rng)]
    net = qs.MLP(max_batch=2048)
    net.set_params(qs.pack_params(P))
    return net


def _box_queries(n, seed):
    """Queries over the box, a tenth of them moved outside it (k = 4.5 or xi = 230)."""
    rng = np.random.default_rng(seed)
    nb = 10 ** rng.uniform(-3, -1, n)
    g = 10 ** rng.uniform(1, 4, n)
    k = rng.uniform(0.05, 4, n)
    xi = rng.uniform(0, 200, n)
    tau = rng.uniform(0, 1, n) * 10 * np.sqrt(g / nb)
    out = rng.random(n) < 0.1
    k[out & (rng.random(n) < 0.5)] = 4.5
    xi[out & (k != 4.5)] = 230.0
    return np.stack([np.log(nb), np.log(g), k, xi, tau], axis=1).astype(np.float32)


def _small_queries():
    """Ten queries in two (n_b, gamma) groups; cheap for the solver of the AUTO mode."""
    rows = []
    for nb, g in [(0.0113, 137.0), (0.047, 310.0)]:
        tf = 10 * math.sqrt(g / nb)
        for k, xi, s in [(0.5, 2.0, 40), (2.0, 2.0, 40), (2.0, 3.3, 30), (3.5, 1.9, 0), (0.5, 0.4, 20)]:
            rows.append([math.log(nb), math.log(g), k, xi, s * tf / 200])
    return np.array(rows, np.float32)


def _table(qs, torch, seed):
    """Random held-out error estimates: trusted (1e-3), too large (0.5) or missing (-1)."""
    rng = np.random.default_rng(seed)
    t = rng.choice(np.array([1e-3, 0.5, -1.0], np.float32), qs.GROWTH_BINS, p=[0.96, 0.02, 0.02])
    return torch.as_tensor(t, device="cuda"), t


def _noalloc(qs, torch, net, table, q):
    n = len(q)
    out = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    flag = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    qs.growth_map_noalloc(net, table, 1e-2, torch.as_tensor(q, device="cuda"), out, flag)
    torch.cuda.synchronize()
    return out.cpu().numpy(), flag.cpu().numpy()


def test_noalloc_matches_growth_map(qs):
    import torch
    net = _net(qs, 11)
    table, htab = _table(qs, torch, 12)
    for n, seed in ((3000, 21), (1200, 22)):          # second call smaller: scratch reused
        q = _box_queries(n, seed)
        out, flag = _noalloc(qs, torch, net, table, q)
        sur = torch.empty(n, dtype=torch.float32, device="cuda")
        qs.growth_map(net, None, 0.0, torch.as_tensor(q, device="cuda"), qs.GROWTH_SURROGATE, sur)
        assert np.array_equal(out, sur.cpu().numpy()), "network answers differ from qs_growth_map"
        # the routing of the AUTO mode itself (its solver answers the flagged queries)
        used = torch.zeros(n, dtype=torch.uint8, device="cuda")
        auto = torch.empty(n, dtype=torch.float32, device="cuda")
        qs.growth_map(net, table, 1e-2, torch.as_tensor(q, device="cuda"), qs.GROWTH_AUTO, auto, used)
        u = used.cpu().numpy()
        assert np.array_equal(flag, u)
        assert np.array_equal(out[u == 0], auto.cpu().numpy()[u == 0])
        assert 0 < flag.sum() < n
    # against the AUTO mode itself (its solver answers the flagged queries)
    q = _small_queries()
    bins = Gr.bin_of(Gr.box_coords(q.astype(np.float64)))
    tz = torch.full((qs.GROWTH_BINS,), 1e-3, dtype=torch.float32, device="cuda")
    tz[int(bins[1])] = 0.5
    tz[int(bins[6])] = -1.0
    out, flag = _noalloc(qs, torch, net, tz, q)
    auto = torch.empty(len(q), dtype=torch.float32, device="cuda")
    used = torch.zeros(len(q), dtype=torch.uint8, device="cuda")
    qs.growth_map(net, tz, 1e-2, torch.as_tensor(q, device="cuda"), qs.GROWTH_AUTO, auto, used)
    u = used.cpu().numpy()
    assert np.array_equal(flag, u) and 0 < u.sum() < len(q)
    assert np.array_equal(out[u == 0], auto.cpu().numpy()[u == 0])
    net.close()


def test_noalloc_rejects_oversize_and_empty(qs):
    import torch
    net = _net(qs, 13)
    L = qs.lib()
    q = torch.zeros((4, 5), dtype=torch.float32, device="cuda")
    out = torch.full((4,), 3.0, dtype=torch.float32, device="cuda")
    flag = torch.zeros(4, dtype=torch.uint8, device="cuda")
    vp = ctypes.c_void_p
    st = L.qs_growth_map_noalloc(net.h, None, ctypes.c_float(1e-2), vp(q.data_ptr()),
                                 ctypes.c_int64(qs.GROWTH_NOALLOC_MAX + 1), vp(out.data_ptr()), vp(flag.data_ptr()))
    assert st == qs.QS_ERR_ARG
    assert b"exceed" in L.qs_last_error()
    st = L.qs_growth_map_noalloc(net.h, None, ctypes.c_float(1e-2), vp(q.data_ptr()), ctypes.c_int64(0),
                                 vp(out.data_ptr()), vp(flag.data_ptr()))
    assert st == qs.QS_OK
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 3.0)
    net.close()
