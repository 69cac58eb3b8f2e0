"""Adversarial channel-weight vectors for the integer allocation N_c = alpha_c N
(largest remainders, ties to the lower channel, floor min_calls).

Inputs only: every case is a (alpha, N) pair built so that the allocation's
integer decisions sit on a knife edge -- remainders exactly tied, remainders
one ulp apart, alpha_c N one ulp from an integer, products that are not
representable (a fused multiply-add would see a different remainder), and
floors that bind.  Seeded, deterministic."""
import numpy as np


def cases(n_cases: int = 300, seed: int = 2024):
    rng = np.random.default_rng(seed)
    out = []
    kinds = ["tied", "ulp_apart", "near_integer", "inexact", "floors", "mixed"]
    for q in range(n_cases):
        kind = kinds[q % len(kinds)]
        K = int(rng.integers(2, 9))
        if kind in ("tied", "ulp_apart", "near_integer"):
            N = int(2 ** rng.integers(8, 16))  # alpha_c N exact: the scaling is by 2^k
        else:
            N = int(rng.choice([1000, 3000, 10_000, 12_345, 99_999, 30, 7 * 11 * 13]))
        N = max(N, 10 * K)
        m = rng.integers(10, max(11, N // K), K).astype(np.float64)
        if kind == "tied":
            f = float(rng.choice([0.25, 0.5, 0.75, 0.125]))
            v = m + f
        elif kind == "ulp_apart":
            f = float(rng.uniform(0.1, 0.9))
            v = m + f
            j = int(rng.integers(0, K))
            v[j] = np.nextafter(v[j], np.inf if rng.random() < 0.5 else -np.inf)
        elif kind == "near_integer":
            v = m.copy()
            for j in range(K):
                r = rng.random()
                if r < 0.4:
                    v[j] = np.nextafter(m[j], -np.inf)
                elif r < 0.8:
                    v[j] = np.nextafter(m[j], np.inf)
        elif kind == "inexact":
            # alpha_c = k_c / D: alpha_c N rounds to (or near) an integer while
            # the exact product does not
            D = int(rng.choice([3, 7, 10, 100, 1000]))
            k = rng.integers(1, D, K)
            out.append((k / D, N, kind))
            continue
        elif kind == "floors":
            v = m.copy()
            for j in range(K):
                if rng.random() < 0.5:
                    v[j] = float(rng.choice([0.0, 1e-300, 3.0, 9.999999999999998, 9.5]))
        else:
            v = m + rng.random(K)
        alpha = v / N
        out.append((alpha, N, kind))
    return out
