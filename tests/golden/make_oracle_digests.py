"""Write tests/golden/oracle_digests.json: the CPU oracle's sketch digest of
whole workload streams that are too long to replay inside a GPU test.

Calls only the oracle and the stream generators.  Run from the repository
root:  python tests/golden/make_oracle_digests.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import streamgen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_digests.json")


def main():
    res = {}
    for i in (0, 1):
        cfg = streamgen.CONFIGS[i]
        V = cfg["V"]
        C = streamgen.ceil_log2(V)
        D = 2 * C
        u, v, d = streamgen.config_stream(i)
        t = time.time()
        sk = oracle.Sketch(V, C, D, cfg["S"])
        sk.apply(u, v)
        dg = sk.digest()
        res[cfg["name"]] = {"V": V, "C": C, "D": D, "S": cfg["S"], "n_updates": int(len(u)),
                            "digest": "0x%016x" % dg}
        print(cfg["name"], res[cfg["name"]], "%.1fs" % (time.time() - t), flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
