"""The oracle's chain on fixed short runs equals the committed digest
(tests/golden/oracle_chain_digest.json, written from the oracle alone by
tests/golden/make_oracle_golden.py): a guard against unintended changes to
the oracle, beside the pins against the paper in the other test_oracle_*
files.  Continuous-field energies are compared to 1e-12 relative (another
libm could round exp differently); everything else exactly."""
import importlib.util
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_oracle_golden",
                                               os.path.join(HERE, "golden", "make_oracle_golden.py"))
gen = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(gen)
DIGEST = json.load(open(gen.DIGEST))


@pytest.mark.parametrize("case", gen.CASES, ids=[c["name"] for c in gen.CASES])
def test_oracle_chain_matches_digest(oracle_mod, case):
    got = gen.run_case(oracle_mod, case)
    want = DIGEST[case["name"]]
    for key in ("R", "spins_sha256", "perm", "counters", "att", "acc", "temps", "magnetizations"):
        assert got[key] == want[key], key
    if case["kind"] == "b":
        assert got["energies"] == want["energies"]
    else:
        for a, b in zip(got["energies"], want["energies"]):
            fa, fb = float.fromhex(a), float.fromhex(b)
            assert abs(fa - fb) <= 1e-12 * max(1.0, abs(fb))


def test_digest_covers_the_interesting_paths():
    """The fixed runs exercise accepted exchanges, an adaptive insertion and
    a call that ends inside an interval."""
    assert any(sum(v["acc"]) > 0 for v in DIGEST.values())
    assert DIGEST["bimodal_l8_adaptive"]["R"] > 4
    assert DIGEST["bimodal_l4_ragged"]["counters"][0] % 5 != 0
