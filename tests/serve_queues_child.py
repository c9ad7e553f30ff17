"""Child process of test_gpu_server_queues: a fresh process whose only
streams are the null stream (the caller's) and the server's three.

Long chains occupy the pipelined and the general queue; then a copy on the
caller's stream, and requests on geometries the server has not built yet
(one for the long-row queue, whose kernel is not running and must be
launched, one for the pipelined queue) must finish within their deadlines.  Every chain is
cancelled and the server destroyed before the process exits, whatever
happened, so every kernel ends.  Prints one JSON line."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import paper_1411_4622_amd as P  # noqa: E402


def main() -> int:
    P.load()
    torch.zeros(1, device="cuda")  # the null stream first
    srv = P.Server(mem_budget=8 << 30)  # default slots, idle time and queues
    out = {"ok": False}
    tickets = []
    try:
        rng = np.random.default_rng(1)

        def request(N, U, dt, M, steps):
            K = int(np.ceil(np.sqrt(2.0) * N))
            ang = np.arange(U) * (180.0 / U)
            yy, xx = np.mgrid[:N, :N] - (N - 1) / 2.0
            mask = (xx * xx + yy * yy <= (N / 2.0) ** 2).astype(np.uint8)
            geom = P.Geometry(N, ang, K, mask, dt)
            sino = torch.from_numpy(rng.random((U, K)) * N * 0.3).cuda()
            img = torch.full((N, N), 0.3, dtype=torch.float64, device="cuda")
            prm = P.SatParams(n_steps=steps, seed=3, chain_id=N + U, m_cand=M, T0=1e-2, TN=1e-6,
                              n_stages=100, precision=dt, resync_every=4096 if dt == "f32" else 0)
            torch.cuda.current_stream().synchronize()
            t = srv.submit(geom, sino, img, prm)
            assert t is not None, "request %dx%d refused" % (N, U)
            return t

        # long chains on the pipelined (rows <= 512) and general (FP64) queues
        for N, U, dt, M in [(256, 180, "f32", 8), (64, 90, "f64", 16)]:
            tickets.append(request(N, U, dt, M, 10**9))
        time.sleep(1.0)
        out["long_running"] = [srv.poll(t) is None for t in tickets]
        # a copy on the caller's stream
        x = torch.ones(16 << 20, device="cuda")
        t0 = time.time()
        y = x.clone()
        ev = torch.cuda.Event()
        ev.record()
        while not ev.query() and time.time() - t0 < 10.0:
            time.sleep(0.001)
        out["copy_s"] = time.time() - t0
        out["copy_done"] = bool(ev.query())
        if out["copy_done"]:
            out["copy_done"] = float(y[-1]) == 1.0
        # requests whose PILAs are built on arrival: 40 x 40 at 720 angles
        # (rows of ~900 entries: the long-row body) and a pipelined one
        for name, (N, U, M) in [("small_long", (40, 720, 4)), ("small_piped", (48, 60, 4))]:
            t0 = time.time()
            t = request(N, U, "f32", M, 2000)
            st = None
            while st is None and time.time() - t0 < 30.0:
                st = srv.poll(t)
                time.sleep(0.002)
            out[name + "_s"] = time.time() - t0
            out[name + "_done"] = st is not None and st["status"] == 0
            out[name + "_body"] = None if st is None else st["body"] & 15
        out["ok"] = True
    finally:
        for t in tickets:
            try:
                srv.cancel(t)
            except Exception:
                pass
        t0 = time.time()
        left = list(tickets)
        while left and time.time() - t0 < 120.0:
            left = [t for t in left if srv.poll(t) is None]
            time.sleep(0.01)
        out["cancelled_s"] = time.time() - t0
        out["left"] = len(left)
        srv.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
