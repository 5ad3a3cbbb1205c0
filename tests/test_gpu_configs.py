"""The N = 2^16 workloads beyond the metric's job, on the benchmark's ring:

* lockstep jobs of the attention-layer shape (Section 5.2, the LLaMA-shaped
  run: 16 ciphertexts per job, 4096 Softmax of dimension 128, logits
  N(0, 4^2) clipped to [-64, 0]): every job's output ciphertexts are the
  same words alone and in the lockstep batch, and each job meets >= 16 bits
  against the FP64 Softmax;
* the paper's own input law (Section 5.2, "Input distribution":
  N(-M/2, (M/6)^2) tail-cut to [-M, 0]) at dimension 256 with M = 128
  (version B, 64 ciphertexts: 8192 Softmax, more than the paper's 5000) and
  M = 256 (Algorithm SM, as in the paper's table for that range: version B's
  main thread needs k + 2 levels after the exponential, one more than the
  twelve user levels leave at k = 6; 8 ciphertexts, 1024 Softmax);
* a small serving mix at full size (dimensions 256, 4096 and 32768, two
  workers): each result the same alone and in the mix, the batches of the
  two workers overlapping in time, and the precision of each dimension;
* large dimensions (8192 and 32768, Algorithm SM on 8 ciphertexts, two
  Newton steps per inverse square root by default): >= 16 bits, and without
  the steps the bound their degree-255 polynomials leave; at 8192 also
  version B, whose last iteration takes the steps."""
import numpy as np
import pytest

import synthetic
from oracle import softmax as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_11184_amd import hs
    c = hs.Context(synthetic.preset("fgb16"), device=0, stream=hs.current_stream())
    c.keygen(2003)
    return c


def test_layer_jobs_in_lockstep(ctx):
    from paper_2410_11184_amd.softmax import encrypt_logits, decrypt_outputs
    g = synthetic.WORKLOADS["fgb16_uneven"]["groups"][0]
    J, n, M, m = 3, g["n"], g["M"], g["m"]
    xs = [synthetic.group_logits("fgb16_uneven", 0, j) for j in range(J)]
    cts = [encrypt_logits(ctx, x, M, seed=4000 + j) for j, x in enumerate(xs)]
    print("layer jobs: %d x %d ciphertexts, n=%d, M=%g" % (J, m, n, M), flush=True)
    together = ctx.softmax([c for cj in cts for c in cj], n, M, variant=1, jobs=J)
    assert len(together) == J * m
    for j in range(J):
        alone = ctx.softmax(cts[j], n, M, variant=1)
        for i in range(m):
            assert np.array_equal(alone[i].export(), together[j * m + i].export()), (j, i)
        bits = S.precision_bits(S.softmax(xs[j]), decrypt_outputs(ctx, together[j * m:(j + 1) * m], n))
        print("job %d: %s" % (j, bits))
        assert bits["worst"] >= 16.0, (j, bits)


@pytest.mark.parametrize("M", [128.0, 256.0])
def test_paper_input_law(ctx, M):
    from paper_2410_11184_amd.softmax import encrypt_logits, decrypt_outputs
    n = 256
    m, variant = (64, 1) if M <= 128 else (8, 0)
    L = m * ctx.slots // n
    x = synthetic.logits_paper(L, n, M, seed=1160 + int(M))
    cts = encrypt_logits(ctx, x, M, seed=5160 + int(M))
    print("paper law: M=%g, %d Softmax of dim %d" % (M, L, n), flush=True)
    y = decrypt_outputs(ctx, ctx.softmax(cts, n, M, variant=variant), n)
    bits = S.precision_bits(S.softmax(x), y)
    print("M=%g: %s, stats %s" % (M, bits, ctx.softmax_stats()))
    assert np.max(np.abs(y.sum(axis=1) - 1.0)) < 2 ** -12
    # M = 128 carries the metric's 16-bit bar; at M = 256 the paper reports
    # 16.6 bits worst case for Algorithm SM (measured here: 18.3)
    assert bits["worst"] >= 16.0, bits


def test_serving_at_full_size():
    from paper_2410_11184_amd import serve
    p = synthetic.preset("fgb16")
    rng = np.random.default_rng(1004)
    mix = []
    for rid, (n, V) in enumerate([(256, 300), (4096, 5), (256, 40), (32768, 1), (4096, 3), (256, 128)]):
        mix.append((rid, synthetic.logits_uniform(V, n, 128.0 if n < 32768 else 256.0, seed=int(rng.integers(1 << 30)))))
    srv = serve.SoftmaxServer(p, workers=2, hbm_budget_gb=120.0, variant=1, key_seed=2004)
    mixed = [srv.submit(rid, x, 128.0 if x.shape[1] < 32768 else 256.0) for rid, x in mix]
    for r in mixed:
        assert r.done.wait(600)
    srv.close()
    assert all(r.error is None for r in mixed), [str(r.error) for r in mixed if r.error]
    assert len({r.worker for r in mixed}) == 2, "one worker did all the work"
    spans = sorted((r.t_start, r.t_done, r.worker) for r in mixed)
    overlap = any(a[2] != b[2] and a[0] < b[1] and b[0] < a[1] for i, a in enumerate(spans) for b in spans[i + 1:])
    assert overlap, "the two workers' batches never overlapped in time"
    alone = serve.SoftmaxServer(p, workers=1, hbm_budget_gb=120.0, variant=1, key_seed=2004)
    worst = {}
    for (rid, x), rm in zip(mix, mixed):
        ra = alone.submit(rid, x, 128.0 if x.shape[1] < 32768 else 256.0)
        assert ra.done.wait(600) and ra.error is None
        assert np.array_equal(ra.result, rm.result), "request %d differs alone and in the mix" % rid
        b = S.precision_bits(S.softmax(x), rm.result)["worst"]
        worst[x.shape[1]] = min(worst.get(x.shape[1], 99.0), b)
    alone.close()
    print("worst bits by dimension:", worst, "latency:", serve.latency_stats(mixed))
    # above n = 2048 two Newton steps per inverse square root: version B's
    # last iteration at 4096, Algorithm SM at 32768 (measured 19.7 and 16.9)
    assert worst[256] >= 16.0, worst
    assert worst[4096] >= 16.0 and worst[32768] >= 15.0, worst


@pytest.mark.parametrize("case", [(200, 128.0, 2, 0), (16, 32.0, 3, 0), (256, 128.0, 2, 1)],
                         ids=["padded-n200", "cube-n16", "newton-n256"])
def test_variants_at_full_size(ctx, case):
    # a dimension that is not a power of two (200, packed as 256),
    # normalize-and-cube (n = 16, where the appendix expects t-th powers to
    # pay: their later intervals [~n^-(t-1), 1] widen with n) and one Newton
    # step per inverse square root (n = 256, first guesses of degrees 31 /
    # 31 / 63), all with Algorithm SM and
    # bootstrapping on the benchmark's ring: one ciphertext each, precision
    # against FP64
    from paper_2410_11184_amd.softmax import encrypt_logits, decrypt_outputs
    n, M, t, nw = case
    n2 = 1 << (n - 1).bit_length()
    L = ctx.slots // n2
    x = synthetic.logits_uniform(L, n, M, seed=1200 + n)
    cts = encrypt_logits(ctx, x, M, seed=5200 + n)
    print("variant: n=%d (packed as %d), M=%g, power %d" % (n, n2, M, t), flush=True)
    kw = dict(inv_degrees=(31, 31, 63)) if nw else {}
    y = decrypt_outputs(ctx, ctx.softmax(cts, n, M, variant=0, power=t, newton_steps=nw, **kw), n)
    bits = S.precision_bits(S.softmax(x), y)
    print("n=%d power %d: %s, stats %s" % (n, t, bits, ctx.softmax_stats()))
    assert y.shape == (L, n)
    assert np.max(np.abs(y.sum(axis=1) - 1.0)) < 2 ** -10
    # Newton (first guesses of degrees 31 / 31 / 63, one step each) is a
    # trade study: reported, held to 12 bits
    assert bits["worst"] >= (12.0 if nw else 16.0), bits


@pytest.mark.parametrize("n", [8192, 32768])
def test_large_dimensions(ctx, n):
    # above n = 2048 the last normalisation polynomial (degree 255, the most
    # the levels allow) cannot resolve [~1/n, 1]; two Newton steps from it,
    # the first guess bootstrapped when the levels run short, square its
    # error twice (measured 19.7 and 17.7 bits)
    from paper_2410_11184_amd.softmax import encrypt_logits, decrypt_outputs
    M = 256.0 if n == 32768 else 128.0
    m = 8
    L = m * ctx.slots // n
    x = synthetic.logits_uniform(L, n, M, seed=6000 + n)
    cts = encrypt_logits(ctx, x, M, seed=6100 + n)
    print("large dimension: n=%d, %d vectors in %d ciphertexts" % (n, L, m), flush=True)
    y = decrypt_outputs(ctx, ctx.softmax(cts, n, M, variant=0), n)
    bits = S.precision_bits(S.softmax(x), y)
    print("n=%d: %s, stats %s" % (n, bits, ctx.softmax_stats()))
    assert bits["worst"] >= 16.0, bits
    y1 = decrypt_outputs(ctx, ctx.softmax(cts, n, M, variant=0, newton_steps=-1), n)
    b1 = S.precision_bits(S.softmax(x), y1)
    print("n=%d without Newton's steps: %s" % (n, b1))
    assert b1["worst"] < bits["worst"] - 4.0, (b1, bits)
    if n <= 16384:
        # version B, the two steps in its last iteration only (measured
        # 20.7 bits at n = 8192, M = 128)
        yb = decrypt_outputs(ctx, ctx.softmax(cts, n, M, variant=1), n)
        bb = S.precision_bits(S.softmax(x), yb)
        print("n=%d version B: %s, stats %s" % (n, bb, ctx.softmax_stats()))
        assert bb["worst"] >= 16.0, bb


@pytest.mark.parametrize("case", [("fgb16_smb64", 256, 128.0, 16, 4), ("fgb16_uneven", 128, 64.0, 16, 8)],
                         ids=["dim256-J4", "layer-J8"])
def test_packed_jobs_at_full_size(ctx, case):
    # version B with the jobs' auxiliary ciphertexts packed (merge = 1): n / m
    # jobs' sums in one auxiliary ciphertext; every job >= 16 bits against
    # its own FP64 Softmax, rows summing to 1, and job 0 within 2^-16 of the
    # same batch run alone (equal to the precision: the shared bootstraps
    # add their own noise)
    from paper_2410_11184_amd.softmax import encrypt_logits, decrypt_outputs
    name, n, M, m, J = case
    L = m * ctx.slots // n
    if name == "fgb16_uneven":
        xs = [synthetic.group_logits(name, 0, j) for j in range(J)]      # the layer jobs' own logits
    else:
        xs = [synthetic.workload_logits(name, L=L, seed=9100 + j) for j in range(J)]
    assert all(x.shape == (L, n) for x in xs)
    cts = [c for j, x in enumerate(xs) for c in encrypt_logits(ctx, x, M, seed=9200 + j)]
    print("packed jobs: %d x %d ciphertexts, n=%d, M=%g" % (J, m, n, M), flush=True)
    out = ctx.softmax(cts, n, M, variant=1, jobs=J, merge=1)
    st = ctx.softmax_stats()
    alone = decrypt_outputs(ctx, ctx.softmax(cts[:m], n, M, variant=1), n)
    for j in range(J):
        y = decrypt_outputs(ctx, out[j * m:(j + 1) * m], n)
        bits = S.precision_bits(S.softmax(xs[j]), y)
        print("job %d: %s" % (j, bits))
        assert bits["worst"] >= 16.0, (j, bits)
        assert np.max(np.abs(y.sum(axis=1) - 1.0)) < 2 ** -12
        if j == 0:
            d = float(np.max(np.abs(y - alone)))
            print("job 0 against alone: 2^%.2f, stats %s" % (np.log2(d + 1e-300), st))
            assert d < 2 ** -16
