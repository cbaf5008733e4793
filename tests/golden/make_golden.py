"""Write tests/golden/oracle_values.json: oracle Torontonians of the seeded
workloads, for the GPU parity tests and the precision report.

Calls only the CPU oracle (oracle/) and the seeded input generator; nothing
here comes from the GPU path.  Each entry records the generator arguments,
the SHA-256 of the O bytes, the oracle mode, its double-double result, the
sum of |t| and the sum of t^2.

Modes: "quad" (__float128 throughout) where it finishes in minutes (n <= 20)
and for one n = 24 seed (about 40 minutes on 8 threads), "f64" (the FP64
floor the GPU's FP64 path shares), and "ld" (x87 extended, 64-bit
significand) as the accurate reference at n = 24 and 30, where __float128
would take hours to days.

    python tests/golden/make_golden.py [--only NAME ...] [--threads T] [--out FILE]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2109_04528_amd import inputs as gen  # noqa: E402

OUT = os.path.join(HERE, "oracle_values.json")

# name -> (n, seed, r_lo, r_hi, eta, mode)
CASES = {}
for s in range(4):
    CASES[f"prec_n16_s{s}"] = (16, s, 0.3, 1.2, 0.9, "quad")
    CASES[f"prec_n20_s{s}"] = (20, s, 0.3, 1.2, 0.9, "quad")
CASES["first_n10_s0"] = (10, 0, 0.5, 1.0, 0.5, "quad")
for s in range(8):
    CASES[f"pair_n24_s{s}"] = (24, s, 0.5, 1.0, 0.7, "f64")
for s in range(8):
    CASES[f"pair_n24_s{s}_ld"] = (24, s, 0.5, 1.0, 0.7, "ld")
# the hardest n = 24 seed (R = 1.2e15) once more in __float128: the extended
# reference's own floor there is about 1e-8 relative
CASES["pair_n24_s3_q"] = (24, 3, 0.5, 1.0, 0.7, "quad")
CASES["prec_n30_s0"] = (30, 0, 0.3, 1.2, 0.9, "f64")
CASES["prec_n30_s0_ld"] = (30, 0, 0.3, 1.2, 0.9, "ld")

MODES = {"quad": orc.QUAD, "f64": orc.F64, "ld": orc.LD}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=OUT, help="where to write (default: oracle_values.json)")
    args = ap.parse_args()
    out = args.out
    data = json.load(open(out)) if os.path.exists(out) else {}
    if not args.only:
        data = {}  # a full run rewrites every entry
    for name, (n, seed, lo, hi, eta, mode) in CASES.items():
        if args.only and name not in args.only:
            continue
        O = gen.random_O(n, seed, lo, hi, eta)
        t0 = time.time()
        r = orc.tor(O, mode=MODES[mode], threads=args.threads)
        dt = time.time() - t0
        data[name] = {"n": n, "seed": seed, "r_lo": lo, "r_hi": hi, "eta": eta, "oracle_mode": mode,
                      "sha256": gen.sha256(O), "tor_hi": r.hi, "tor_lo": r.lo, "sum_abs": r.sum_abs,
                      "sum_sq": r.sum_sq, "subsets": r.count, "seconds": round(dt, 1)}
        print(f"{name}: {r.value!r} R={r.cancellation:.3e} ({dt:.1f} s)", flush=True)
        with open(out + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    main()
