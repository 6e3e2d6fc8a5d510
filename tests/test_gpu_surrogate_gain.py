"""What the trained surrogate gains over the method without it -- the solver answering every
growth-map query -- end to end on the GPU at a reduced size.

Training examples come from a 32-instance uniform-seed sweep, held-out examples from a
second sweep and check examples from a third (solver, growth targets and example draws all
in the library's kernels); the network is trained by the library's own forward, backward and
AdamW kernels.  The gain, stated as assertions:
  - accuracy: after training, the held-out RMS error is below a tenth of what the best
    constant (the targets' mean) and the untrained network give;
  - the held-out error table keeps its promise out of sample: of the check sweep's examples
    in the bins that the table trusts at a tolerance, at least 90 % are within it (the
    table holds a per-bin 99th percentile);
  - speed: the network answers scattered box queries more than 100 times faster per query
    than the solver does.
"""
import time

import numpy as np
import pytest

from oracle import growth as Gr

pytestmark = pytest.mark.gpu


def test_trained_network_gain_over_solver(qs):
    import torch
    from paper_2607_24234_amd import surrogate as S

    X, T = S.examples(S.sweep_instances(n_instances=32, seed=10), 1 << 19, 11)
    Xh, Th = S.examples(S.sweep_instances(n_instances=32, seed=12), 1 << 18, 13)
    Xc, Tc = S.examples(S.sweep_instances(n_instances=32, seed=14), 1 << 18, 15)
    t = T.cpu().numpy().astype(np.float64)
    th = Th.cpu().numpy().astype(np.float64)
    net = qs.MLP(max_batch=1 << 16)
    net.set_params(qs.pack_params(S.initial_params(3, float(t.mean()), float(t.std()))))

    rms_const = float(np.sqrt(np.mean((th - t.mean()) ** 2)))
    rms_init = S.held_out_errors(net, Xh, Th)["rms"]
    S.train(net, X, T, epochs=12, batch=8192, lr=1e-3)
    err = S.held_out_errors(net, Xh, Th)
    print("held-out rms: constant %.4f, untrained %.4f, trained %.4f (p99 %.4f)"
          % (rms_const, rms_init, err["rms"], err["p99"]))
    assert err["rms"] < 0.1 * rms_const and err["rms"] < 0.1 * rms_init

    # the error table from the held-out sweep, checked on the third sweep
    table = S.calibrate(net, Xh, Th).cpu().numpy()
    known = table[table >= 0]
    assert known.size > 0
    tol = float(np.median(known))
    yc = net.forward(Xc).cpu().numpy().astype(np.float64)
    ec = np.abs(yc - Tc.cpu().numpy())
    trusted = (table >= 0) & (table <= tol)
    inb = trusted[Gr.bin_of(Xc.cpu().numpy())]
    cover = float(np.mean(ec[inb] <= tol))
    print("tolerance %.4f: %d of %d bins trusted, %.1f %% of check examples there, %.2f %% of those within"
          % (tol, int(trusted.sum()), known.size, 100 * inb.mean(), 100 * cover))
    assert inb.mean() > 0.05 and cover >= 0.9

    # speed on scattered queries from the box
    q = torch.as_tensor(S.query_box(1 << 20, 16), device="cuda")
    out = torch.empty(q.shape[0], device="cuda")
    qs.growth_map(net, None, 0.0, q, qs.GROWTH_SURROGATE, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4):
        qs.growth_map(net, None, 0.0, q, qs.GROWTH_SURROGATE, out)
    torch.cuda.synchronize()
    s_net = (time.perf_counter() - t0) / (4 * q.shape[0])
    n_s = 16
    t0 = time.perf_counter()
    qs.growth_map(None, None, 0.0, q[:n_s], qs.GROWTH_SOLVER, out[:n_s])
    torch.cuda.synchronize()
    s_sol = (time.perf_counter() - t0) / n_s
    print("per query: network %.3e s, solver %.3e s (%.2e x)" % (s_net, s_sol, s_sol / s_net))
    assert s_sol > 100.0 * s_net
