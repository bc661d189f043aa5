"""Shot-simulation serving with continuous batching.

Requests (one seismic shot each: grid size, layered medium, source, 128
receivers, step count) arrive over time.  The server keeps every admitted
shot's state resident in HBM, admits new shots whenever a slot and the memory
budget allow (footprint = the shot workspace reported by the library plus its
trace buffer), and advances all active shots together: each tick is k time
steps in batched launches of several steps each (as lb_blocked_steps gives),
replayed from a captured HIP graph.  A shot that reaches its last step stops
updating inside the tick; once the tick has run, its traces are copied out
and its slot and memory are freed.

run_sequential() is the baseline on the same trace: one shot at a time,
picked by the same admission policy, through the single-grid lb_step_n path
(several steps per launch, one shot per launch).

Latency of a request = completion - arrival = queue wait + service.
"""
import argparse
import collections
import json
import sys
import time

import numpy as np


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def summarize(records, wall):
    lat = [r["done"] - r["arrival"] for r in records]
    wait = [r["admit"] - r["arrival"] for r in records]
    svc = [r["done"] - r["admit"] for r in records]
    lups = sum(r["n"] * r["n"] * r["nsteps"] for r in records)
    return {
        "completed": len(records), "wall_s": round(wall, 3),
        "shots_per_s": round(len(records) / wall, 3) if wall > 0 else None,
        "GLUPS": lups / wall / 1e9 if wall > 0 else None,
        "latency_p50_s": _pct(lat, 50), "latency_p99_s": _pct(lat, 99),
        "wait_p50_s": _pct(wait, 50), "wait_p99_s": _pct(wait, 99),
        "service_p50_s": _pct(svc, 50), "service_p99_s": _pct(svc, 99),
    }


def _cost_s(req, rate):
    """Estimated service time of a request alone on the GPU (seconds)."""
    return req["n"] * req["n"] * req["nsteps"] / rate


def _pick_order(queue, policy, now, rate, aging):
    """Queue order for admission.  fifo: arrival order.  sjf: shortest
    estimated service first, with aging: a request's key is s - aging * w
    for service estimate s and queue wait w (seconds), so a large request
    that has waited long enough goes before fresh small ones instead of
    starving under overload."""
    if policy == "fifo":
        return sorted(queue, key=lambda r: r["arrival"])
    return sorted(queue, key=lambda r: (_cost_s(r, rate) - aging * max(0.0, now - r["arrival"]), r["arrival"]))


class ShotServer:
    """Continuous-batching server over the lb_batch executor.

    Admission: requests are taken from the queue in the policy's order
    (fifo: arrival; sjf: shortest estimated service first, aged) while a
    slot is free, the memory footprint fits the budget and the active
    lattice nodes stay under node_cap (so that shots are not slowed down by
    too many batch mates: the step cost is proportional to the nodes).  Each
    tick is sized to about tick_ms of GPU work at rate_lups.  The host keeps
    two ticks in flight: it enqueues the next tick while the GPU runs the
    current one, admits new shots without waiting for the ticks, and retires
    a shot once the tick that finished it has completed (lb_batch_completed).
    """

    def __init__(self, budget_bytes=64 << 30, max_slots=32, tick_steps=None,
                 precision="f32", use_graph=True, keep_traces=False, batch=None,
                 policy="sjf", node_cap=4096 * 4096, tick_ms=20.0, rate_lups=4.0e11, aging=0.05):
        import torch
        from . import lbwave
        self.torch = torch
        self.lbwave = lbwave
        # `batch` lets a caller supply an executor with the lbwave.Batch
        # interface (the admission logic is tested on the CPU that way)
        self.batch = batch if batch is not None else lbwave.Batch(
            max_slots, lattice=5, collision="bgk", precision=precision, tau=0.5, use_graph=use_graph)
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.k_fixed = None if tick_steps is None else int(tick_steps)
        self.keep = keep_traces
        self.elem = 8 if precision == "f64" else 4
        self.policy = policy
        self.node_cap = int(node_cap)
        self.tick_ms = float(tick_ms)
        self.rate = float(rate_lups)
        self.aging = float(aging)

    def desc(self, req):
        return self.lbwave.shot_desc(req["n"], req["n"], req["src"], req["nsteps"], req["nrec"],
                                     req["sponge"], 0.1)

    def footprint(self, req):
        d = self.desc(req)
        return self.batch.shot_bytes(d) + req["nrec"] * (req["nsteps"] + 1) * self.elem

    def _admit(self, req):
        from . import inputs
        c = inputs.serving_speed_torch(req, self.batch.device)
        return self.batch.add(self.desc(req), c * c, inputs.serving_wavelet(req),
                              inputs.serving_receivers(req))

    def _tick_steps(self, nodes):
        if self.k_fixed is not None:
            return self.k_fixed
        return int(max(16, min(512, self.tick_ms * 1e-3 * self.rate / max(nodes, 1))))

    def run(self, trace, progress=False):
        """Serve a list of requests (arrival in seconds from the start);
        returns (records, summary).  progress: a line on stderr every 100
        completed shots."""
        pending = collections.deque(sorted(trace, key=lambda r: r["arrival"]))
        queue = []
        active = {}           # slot -> record
        used = 0
        nodes = 0
        done = []
        traces = {}
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while pending or queue or active:
            tn = now()
            while pending and pending[0]["arrival"] <= tn:
                queue.append(pending.popleft())
            if queue and len(active) < self.max_slots:
                queue = _pick_order(queue, self.policy, tn, self.rate, self.aging)
                while queue and len(active) < self.max_slots:
                    req = queue[0]
                    fp = self.footprint(req)
                    nn = req["n"] * req["n"]
                    if active and (used + fp > self.budget or nodes + nn > self.node_cap):
                        break                      # wait for memory / GPU share
                    queue.pop(0)
                    slot = self._admit(req)
                    used += fp
                    nodes += nn
                    active[slot] = {"rid": req["rid"], "arrival": req["arrival"], "admit": now(),
                                    "n": req["n"], "nsteps": req["nsteps"], "bytes": fp, "nodes": nn}
            # retire the shots whose last tick has run
            if active:
                comp = self.batch.completed()
                for slot in list(active):
                    rec = active[slot]
                    if comp[slot] >= rec["nsteps"]:
                        tr = self.batch.remove(slot)
                        if self.keep:
                            traces[rec["rid"]] = tr.cpu().numpy()
                        rec["done"] = now()
                        used -= rec["bytes"]
                        nodes -= rec["nodes"]
                        done.append(active.pop(slot))
                        if progress and len(done) % 100 == 0:
                            print("batched: %d done at %.1f s" % (len(done), now()), file=sys.stderr, flush=True)
            if not active:
                if pending and not queue:
                    time.sleep(max(0.0, min(0.01, pending[0]["arrival"] - now())))
                continue
            times = self.batch.times()
            if self.batch.in_flight() < 2 and any(times[s] < r["nsteps"] for s, r in active.items()):
                self.batch.tick(self._tick_steps(nodes))   # the next tick while one runs
                continue
            if not self.batch.wait_oldest():
                time.sleep(0.0002)
        wall = max(r["done"] for r in done) - min(r["arrival"] for r in done) if done else 0.0
        self.traces = traces
        return done, summarize(done, wall)

    def close(self):
        self.batch.close()


def run_sequential(trace, policy="fifo", precision="f32", keep_traces=False, progress=False,
                   rate_lups=4.0e11, aging=0.05):
    """Baseline: one shot at a time through the single-grid lb_step_n path
    (several steps per launch, no batching), the next shot chosen among the
    arrived requests by the same policy as the batched server."""
    import torch
    from . import inputs, lbwave
    done = []
    traces = {}
    pending = collections.deque(sorted(trace, key=lambda r: r["arrival"]))
    queue = []
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    while pending or queue:
        while pending and pending[0]["arrival"] <= now():
            queue.append(pending.popleft())
        if not queue:
            time.sleep(max(0.0, min(0.01, pending[0]["arrival"] - now())))
            continue
        req = _pick_order(queue, policy, now(), rate_lups, aging)[0]
        queue.remove(req)
        admit = now()
        n = req["n"]
        g = lbwave.Grid(n, n, lattice=5, collision="bgk", precision=precision, tau=0.5,
                        sponge_width=req["sponge"], sponge_sigma_max=0.1,
                        trace_capacity=req["nsteps"] + 1, max_receivers=req["nrec"])
        c = inputs.serving_speed_torch(req, g.device)
        g.set_medium(c * c)
        g.set_source(req["src"][0], req["src"][1], inputs.serving_wavelet(req))
        tr = g.record(inputs.serving_receivers(req), fields=("p",))
        g.step(req["nsteps"])
        g.sync()
        if keep_traces:
            traces[req["rid"]] = tr[0].cpu().numpy()
        done.append({"rid": req["rid"], "arrival": req["arrival"], "admit": admit, "done": now(),
                     "n": n, "nsteps": req["nsteps"]})
        if progress and len(done) % 100 == 0:
            print("one shot per launch: %d done at %.1f s" % (len(done), now()), file=sys.stderr, flush=True)
        g.close()
        del g, tr
    wall = max(r["done"] for r in done) - min(r["arrival"] for r in done) if done else 0.0
    run_sequential.traces = traces
    return done, summarize(done, wall)


def run_fifo(trace, precision="f32", keep_traces=False, progress=False):
    """One shot at a time in arrival order (run_sequential with fifo)."""
    out = run_sequential(trace, "fifo", precision, keep_traces, progress)
    run_fifo.traces = run_sequential.traces
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--tick", type=int, default=None, help="fixed steps per tick (default: adaptive)")
    ap.add_argument("--policy", choices=("fifo", "sjf"), default="sjf")
    ap.add_argument("--node-cap", type=int, default=4096 * 4096)
    ap.add_argument("--mode", choices=("batch", "sequential", "both"), default="both")
    args = ap.parse_args(argv)
    import torch
    from . import inputs
    torch.cuda.set_device(0)
    trace = inputs.serving_trace(args.requests, args.rate, args.seed)
    out = {"requests": args.requests, "rate": args.rate, "seed": args.seed,
           "budget_gb": args.budget_gb, "slots": args.slots, "tick": args.tick,
           "policy": args.policy, "node_cap": args.node_cap}
    if args.mode in ("batch", "both"):
        srv = ShotServer(int(args.budget_gb * (1 << 30)), args.slots, args.tick,
                         policy=args.policy, node_cap=args.node_cap)
        _, out["batched"] = srv.run(trace, progress=True)
        srv.close()
        print("batched", json.dumps(out["batched"]), file=sys.stderr, flush=True)
    if args.mode in ("sequential", "both"):
        _, out["one_shot_per_launch"] = run_sequential(trace, args.policy, progress=True)
        print("one shot per launch", json.dumps(out["one_shot_per_launch"]), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
