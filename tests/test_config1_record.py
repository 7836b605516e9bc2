"""The [[72,12,6]] workload decoded by the double oracle alone (code
capacity p = 0.05, 10^4 shots, |Phi| = 4): the record committed under
tests/golden (counts, logical error rate and its Wilson 95% interval) is
reproduced exactly."""
import os

from tests.golden import make_config1_record as rec


def test_config1_record_reproduces():
    want = {}
    with open(rec.OUT) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, val = line.split(None, 1)
            want[key] = float(val) if "." in val or "e" in val else int(val)
    got = rec.record()
    assert set(got) == set(want)
    for key, val in got.items():
        assert val == want[key], key
    assert want["wilson95_lo"] <= want["ler"] <= want["wilson95_hi"]
    assert want["converged"] <= want["shots"] and want["failed_first_bp"] > 0
