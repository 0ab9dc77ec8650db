"""Write the oracle's expected values for the large workloads (the oracle takes minutes there).

Calls only ``oracle/`` (and ``synth.py`` for bit packing).  For each case it stores, from the FP64
oracle: every environment log-norm lambda_r = ln ||E_r||_2 and ln Z_TN (Sec. II B), and a few
oracle-drawn proposals (Sec. II A-B, Eqs. (4)-(6)) with their bit-packed spins, FP64 log q and
exact energies (Eq. (10)), so that the GPU can build the same realization and evaluate the same
configurations with its teacher-forced log q.  Slices of the largest lattice keep only the first
rows built (from the bottom).

Usage:  python tests/golden/make_oracle_goldens.py [case ...]   (all cases by default; each
        case runs in its own process, BLAS limited to one thread)
"""
import json
import math
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))

# name: (L, chi, p, coupling seed = realization id, proposals K, rows (None = full build))
CASES = {
    "rbim16_s0": (16, 16, 0.109, 0, 4, None),
    "rbim64_s0": (64, 32, 0.109, 0, 4, None),
    "rbim256_p0.10_s0": (256, 48, 0.10, 0, 3, None),
    "rbim256_p0.109_s77": (256, 48, 0.109, 77, 3, None),
    "rbim256_p0.12_s11": (256, 48, 0.12, 11, 3, None),
    "mixed_L128_s14": (128, 32, 0.109, 14, 3, None),
    "mixed_L256_s19": (256, 32, 0.109, 19, 3, None),
    "rbim1024_s0_rows8": (1024, 64, 0.109, 0, 0, 8),
    "rbim1024_s1_rows8": (1024, 64, 0.109, 1, 0, 8),
}
PHILOX_SEED = 0      # proposal stream key of the stored proposals (first proposal id 0)


def path(name):
    return os.path.join(HERE, f"oracle_{name}.json")


def run_case(name):
    sys.path.insert(0, ROOT)
    import numpy as np

    import synth
    from oracle import energy, envbuild, instance, sampler

    L, chi, p, seed, K, rows = CASES[name]
    beta = instance.nishimori_beta(p)
    Jh, Jv = instance.couplings(seed, L, p)
    t0 = time.time()
    env = envbuild.build_env(Jh, Jv, beta, chi, rows=rows)
    t1 = time.time()
    out = {
        "_about": ("FP64 oracle values written by tests/golden/make_oracle_goldens.py (calls only "
                   "oracle/): environment log-norms lambda_r = ln ||E_r||_2 and ln Z_TN "
                   "(Sec. II B), oracle-drawn proposals with FP64 log q (Eqs. (4)-(6)) and exact "
                   "energies (Eq. (10))."),
        "L": L, "chi": chi, "p": p, "beta": beta, "coupling_seed": seed,
        "rows_built": rows if rows is not None else L - 1,
        "lognorm": [float(x) if math.isfinite(x) else None for x in env["lognorm"]],
        "sensitivity_fp32": envbuild.sensitivity(env, 6e-8),
        "oracle_build_s": round(t1 - t0, 1),
    }
    if rows is None:
        out["lnZ"] = float(env["lnZ"])
    if K > 0:
        res = sampler.run(env, Jh, Jv, beta, K=K, seed=PHILOX_SEED, realization=seed,
                          first_proposal=0)
        words = synth.pack_rows(res["spins"])                  # (K, L, W)
        out["proposals"] = {
            "philox_seed": PHILOX_SEED, "realization": seed, "first_proposal": 0,
            "spins_hex": [[" ".join(f"{int(w):016x}" for w in row) for row in words[k]]
                          for k in range(K)],
            "logq": [float(x) for x in res["logq"]],
            "E": [int(x) for x in energy.energy(res["spins"], Jh, Jv)],
            "fallbacks": int(res["fallbacks"]),
        }
        out["oracle_sample_s"] = round(time.time() - t1, 1)
    with open(path(name), "w") as f:
        json.dump(out, f, indent=0)
    print(f"{name}: build {t1 - t0:.1f} s", flush=True)


def main(names):
    if len(names) == 1:
        run_case(names[0])
        return
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), n], env=env)
             for n in names]
    rc = [p.wait() for p in procs]
    if any(rc):
        raise SystemExit(f"failed: {[n for n, r in zip(names, rc) if r]}")


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
