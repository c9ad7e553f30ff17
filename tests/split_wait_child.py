"""Child of test_gpu_split: one split chain under the wait limit the parent
puts in PILA_SPLIT_WAIT_MS; prints its status and body."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

import torch  # noqa: E402

import paper_1411_4622_amd as P  # noqa: E402
from test_gpu_sat import _slice  # noqa: E402


def main():
    P.load()
    N, U, K, M = 48, 600, 68, 32
    sl = _slice(N, U, K, seed=N + U, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=2000, seed=5, chain_id=M, n_stages=40, m_cand=M, T0=None,
                      q_auto=50, delta_max=0.05)
    pl = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, "f64"))
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st, _ = P.sat_run(pl, torch.from_numpy(sl.sino).cuda(), prm, img)
    torch.cuda.synchronize()
    print("status %d %d" % (st["status"], st["body"]), flush=True)


if __name__ == "__main__":
    main()
