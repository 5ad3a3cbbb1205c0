"""Autotuner: interchangeable kernels give identical ciphertexts.

The metric's batched Softmax job (64 ciphertexts, N = 2^16) is run with the
default kernels, then with tuning enabled (each launch shape times its
candidates on scratch data), then with every decision forced to a
non-default candidate (matrix-core base conversion, conversion targets split
over threads, other NTT row orders, batched launches and 8-column tiles): all
three give the same output ciphertexts bit for bit."""
import json

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


def test_tuned_and_forced_variants_match_defaults(tmp_path):
    from paper_2410_11184_amd import hs
    from paper_2410_11184_amd.softmax import encrypt_logits
    w = synthetic.WORKLOADS["fgb16_smb64"]
    ctx = hs.Context(synthetic.preset("fgb16"))
    ctx.keygen(77)
    n, M = w["n"], w["M"]
    L = w["m"] * ctx.slots // n
    cts = encrypt_logits(ctx, synthetic.workload_logits("fgb16_smb64", L=L), M, seed=78)
    try:
        hs.tune_clear()
        hs.tune_enable(False)
        ref = [c.export() for c in ctx.softmax(cts, n, M, variant=1)]
        hs.tune_enable(True)
        tuned = ctx.softmax(cts, n, M, variant=1)
        assert all(np.array_equal(a, b.export()) for a, b in zip(ref, tuned))
        rep = hs.tune_report()
        assert rep, "no shape was tuned"
        for r in rep:
            assert r["us"][r["choice"]] >= 0, r
        kinds = {r["key"].split()[0] for r in rep}
        assert kinds == {"conv", "ntt"}
        print("tuned:", json.dumps(rep[:3]), "... %d entries" % len(rep))
        # force a valid non-default candidate on every shape, cycling through
        # them so that each one is exercised
        forced = []
        for i, r in enumerate(rep):
            alts = [name for name, t in r["us"].items() if t >= 0 and name not in ("valu", "prime-major")]
            forced.append({"key": r["key"], "choice": alts[i % len(alts)] if alts else r["choice"]})
        chosen = {f["choice"] for f in forced}
        for name in ("mfma", "valu/split2", "valu/split4", "storage-order/batched", "prime-major/tile8",
                     "storage-order/tile8"):
            assert name in chosen, name
        path = tmp_path / "forced.json"
        path.write_text("".join(json.dumps(f) + "\n" for f in forced))
        hs.tune_enable(False)
        hs.tune_clear()
        assert hs.tune_load(path) == len(forced)
        out = ctx.softmax(cts, n, M, variant=1)
        for i, (a, b) in enumerate(zip(ref, out)):
            assert np.array_equal(a, b.export()), "ciphertext %d differs under forced variants" % i
    finally:
        hs.tune_enable(False)
        hs.tune_clear()
