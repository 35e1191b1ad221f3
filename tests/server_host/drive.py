"""Drive the served-mode harness library through the Python binding, as the served
benchmark does: one submitter thread queues every request of the trace at once, then
the main thread waits for them in ticket order and releases each.  Exits non-zero on
any error.  Usage: python drive.py LIBHARNESS MAX_INFLIGHT N_REQUESTS ROUNDS"""
import os
import sys
import threading

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from paper_1311_0059_amd import _native as N  # noqa: E402

N.load(sys.argv[1])  # the stand-in library, in place of libaggx.so

import paper_1311_0059_amd as P  # noqa: E402
from datagen import workloads  # noqa: E402


def main():
    inflight, n_req, rounds = int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4])
    reqs = workloads.served_mix(n_req)
    specs = [P.make_spec(16, [(0, "u64")], list(workloads.AGGS_R16_ALL), budget=w.budget) for w in reqs]
    for r in range(rounds):
        srv = P.Server(64 << 30, max_inflight=inflight)
        tickets = [None] * len(reqs)

        def submitter():
            for i, w in enumerate(reqs):
                tickets[i] = srv.submit(specs[i], 0x1000, w.n)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        for i, w in enumerate(reqs):
            res, info = srv.wait(tickets[i])
            assert int(res.n_rows) == min(w.n, 4096) and info["stats"]["records_in"] == w.n, i
            srv.release(tickets[i])
        st = srv.stats()
        assert st["pool_in_use"] == 0 and st["peak_running"] <= inflight, st
        srv.close()
        print(f"round {r}: peak {st['peak_running']} in flight", flush=True)
    print("python driver ok", flush=True)


if __name__ == "__main__":
    main()
