"""Writes tests/golden/broadband_floor.json: the oracle's own round-off floor on the broadband
parity cases (tests/broadband_cases.py), i.e. the element-wise differences between the oracle
and a second numerical route through the same algorithm (tests/oracle_routes.py) from the same
inputs, at every checkpoint of every case.  Uses only oracle/, synth/ and the test-side route.

The GPU tests take max(stated bar, 3 x floor) per metric and checkpoint as their tolerance, so an
element-wise comparison is never asked to be tighter than the oracle can certify itself.

    python tests/golden/make_broadband_floor.py [--jobs 8] [case ...]   (about 25 minutes)
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "broadband_floor.json")


def run_case(name):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from oracle import channel as ch
    from tests import broadband_cases as bc
    from tests.oracle_routes import second_route, second_route_matrices

    t0 = time.perf_counter()

    def trajectory(second):
        env = ch.Env(bc.config(name))
        if second:
            second_route_matrices(env.S)
        env.set_state(bc.initial_state(env.S, bc.CASES[name]["seed"]))
        out = []
        for k, n in enumerate(bc.CASES[name]["steps"]):
            res = env.step(bc.action(name, k, env.S), n)
            out.append((env.state.copy(), res))
        return out

    ref = trajectory(False)
    with second_route():
        alt = trajectory(True)
    floors = {}
    for cp, (a, b) in zip(bc.checkpoints(name), zip(alt, ref)):
        e = bc.state_errors(a[0], b[0])
        e.update(bc.output_errors(a[1], b[1]))
        floors[str(int(cp))] = e
    print(f"  {name}: {time.perf_counter() - t0:.0f} s", flush=True)
    return name, floors


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    jobs = 8
    if "--jobs" in sys.argv:
        jobs = int(sys.argv[sys.argv.index("--jobs") + 1])
        args = [a for a in args if a != str(jobs)]
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from tests import broadband_cases as bc
    names = args or list(bc.CASES)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        for name, floors in ex.map(run_case, names):
            data[name] = floors
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
