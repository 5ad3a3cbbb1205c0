"""Seeded synthetic inputs and parameter presets shared by the tests, the
oracle checks and ``bench.py``.

This module holds no arithmetic of the method: only configuration numbers
(ring degree, prime bit sizes, digit size, secret weight) and numpy draws of
logits.  Both the HIP library and the CPU oracle receive these values as
plain inputs.

Input recipes (Section 5.2, "Input distribution"): the paper draws logits from
a normal law centred at -M/2 with standard deviation M/6, tail-cut to
[-M, 0], and reports that the uniform law on [-M, 0] behaves the same.  The
workload presets below add the shapes of the benchmark configurations.
"""
import numpy as np

# ---------------------------------------------------------------------------
# Parameter presets.  Bit sizes are targets: each prime is the next unused
# prime p = 1 (mod 2N) closest to 2^bits (candidates 2^bits + 1 + j*2N for
# j = 1, -1, 2, -2, ...).  q[0] is the base prime, q[1..user_top] the user
# levels, the rest the bootstrap levels (slot-to-coefficient, modular
# reduction, coefficient-to-slot from bottom to top).
# ---------------------------------------------------------------------------
PRESETS = {
    # Toy, insecure: N = 2^12, 24 Q primes of 40 bits, 2 special primes of
    # 60 bits, digits of 2 primes, scale 2^40, uniform ternary secret.
    "toy12": dict(
        logN=12,
        q_bits=[40] * 24,
        p_bits=[60] * 2,
        digit=2,
        hamming=0,          # 0 = uniform ternary
        log_scale=40,
        user_top=23,
        boot=None,
    ),
    # N = 2^16, scale 2^40, sparse ternary secret of weight 192, digits of 8
    # primes (dnum = 4, P 2^60 above the largest digit), twelve user levels
    # above q0, full-slot bootstrapping.  K = 30 bounds the overflow I of
    # ModRaise (a sum of 193 centred uniforms, standard deviation 4.0):
    # |I| >= 31 has probability below 2^-30 per bootstrap over 2^16
    # coefficients.  The modular reduction approximates exp(2 pi i (K+1) u /
    # 2^3) with degree 63 and squares three times (the same 11 levels as
    # degree 31 and four squarings, whose approximation error at this K
    # would cost about 5 bits of bootstrapping precision).
    "fgb16": dict(
        logN=16,
        q_bits=[53] + [40] * 12 + [40] * 3 + [60] * 11 + [60] * 3,
        p_bits=[60] * 9,
        digit=8,
        hamming=192,
        log_scale=40,
        user_top=12,
        boot=dict(stc_levels=3, evalmod_levels=11, cts_levels=3,
                  K=30, double_angle=3, cos_degree=63, log_boot_scale=60),
    ),
    # Small ring with the same bootstrapping structure, for fast tests.
    "boot10": dict(
        logN=10,
        q_bits=[53] + [40] * 4 + [40] * 3 + [60] * 11 + [60] * 3,
        p_bits=[59] * 8,
        digit=7,
        hamming=64,
        log_scale=40,
        user_top=4,
        boot=dict(stc_levels=3, evalmod_levels=11, cts_levels=3,
                  K=30, double_angle=3, cos_degree=63, log_boot_scale=60),
    ),
    # the same bootstrapping ring with 10 user levels: room for a whole
    # Softmax schedule (with bootstraps) at test size
    "boot10u": dict(
        logN=10,
        q_bits=[53] + [40] * 10 + [40] * 3 + [60] * 11 + [60] * 3,
        p_bits=[59] * 8,
        digit=7,
        hamming=64,
        log_scale=40,
        user_top=10,
        boot=dict(stc_levels=3, evalmod_levels=11, cts_levels=3,
                  K=30, double_angle=3, cos_degree=63, log_boot_scale=60),
    ),
}

SIGMA = 3.2


def preset(name):
    p = dict(PRESETS[name])
    p["N"] = 1 << p["logN"]
    p["slots"] = p["N"] // 2
    p["sigma"] = SIGMA
    return p


# ---------------------------------------------------------------------------
# Logits.  Seeds: numpy PCG64(1000 + workload index) unless given.
# ---------------------------------------------------------------------------
def logits_uniform(L, n, M, seed):
    """L vectors of dimension n, i.i.d. uniform on [-M, 0]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return -M * rng.random((L, n))


def logits_clipped_normal(L, n, M, sigma, seed):
    """N(0, sigma^2) clipped to [-M, 0] (ties at 0 are kept)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.clip(rng.normal(0.0, sigma, size=(L, n)), -M, 0.0)


def logits_paper(L, n, M, seed):
    """The paper's law: N(-M/2, (M/6)^2), tail-cut to [-M, 0] by rejection."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = rng.normal(-M / 2.0, M / 6.0, size=(L, n))
    bad = (out < -M) | (out > 0)
    while bad.any():
        out[bad] = rng.normal(-M / 2.0, M / 6.0, size=int(bad.sum()))
        bad = (out < -M) | (out > 0)
    return out


WORKLOADS = {
    # plain method, toy parameters: 128 Softmax of dim 16, logits U[-8, 0]
    "toy12_sm": dict(preset="toy12", n=16, M=8.0, m=1, L=128, law="uniform", seed=1000),
    # plain method with bootstrapping: 128 Softmax of dim 256, N(0,16^2) clipped to [-128,0]
    "fgb16_sm": dict(preset="fgb16", n=256, M=128.0, m=1, L=128, law="clipped", sigma=16.0, seed=1001),
    # batched: 64 ciphertexts, 8192 Softmax of dim 256, U[-128, 0]
    "fgb16_smb64": dict(preset="fgb16", n=256, M=128.0, m=64, L=8192, law="uniform", seed=1002),
    # uneven batch: attention-score shapes of 32 layers x 32 heads x 128 queries
    # (each layer 4096 Softmax of dim 128 in 16 ciphertexts, N(0,4^2) clipped to
    # [-64, 0]) plus one Softmax of dim 32768 filling a ciphertext, U[-256, 0]
    "fgb16_uneven": dict(preset="fgb16", seed=1003, groups=[
        dict(jobs=32, n=128, M=64.0, m=16, L=4096, law="clipped", sigma=4.0, variant=1),
        dict(jobs=1, n=32768, M=256.0, m=1, L=1, law="uniform", variant=0),
    ]),
    # serving: Poisson arrivals, dimensions log-uniform over 64..32768, 1-512
    # vectors per request, logits U[-128, 0]
    "fgb16_serve": dict(preset="fgb16", seed=1004, count=12, rate=1.0, M=128.0),
}


def serve_stream(count, rate, seed=1004, dims=tuple(2 ** e for e in range(6, 16)), vmax=512, M=128.0):
    """Poisson request stream: (arrival time, dimension, logits) with
    dimensions log-uniform over `dims`, 1..vmax vectors, logits U[-M, 0]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(dims[rng.integers(0, len(dims))])
        V = int(rng.integers(1, vmax + 1))
        out.append((t, n, logits_uniform(V, n, M, seed * 1000 + i)))
    return out


def group_logits(name, gi, job):
    """Logits of job `job` of group `gi` of a multi-group workload."""
    w = WORKLOADS[name]
    g = w["groups"][gi]
    seed = w["seed"] * 1000 + gi * 100 + job
    if g["law"] == "uniform":
        return logits_uniform(g["L"], g["n"], g["M"], seed)
    return logits_clipped_normal(g["L"], g["n"], g["M"], g["sigma"], seed)


def workload_logits(name, L=None, seed=None):
    w = WORKLOADS[name]
    L = w["L"] if L is None else L
    seed = w["seed"] if seed is None else seed
    if w["law"] == "uniform":
        return logits_uniform(L, w["n"], w["M"], seed)
    if w["law"] == "clipped":
        return logits_clipped_normal(L, w["n"], w["M"], w["sigma"], seed)
    return logits_paper(L, w["n"], w["M"], seed)
