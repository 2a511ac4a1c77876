"""The oracle against its own frozen outputs (tests/golden/nested32_oracle.json,
written by tests/golden/make_golden.py, which calls only the oracle): guards
against unnoticed drift of the reference's arithmetic."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_nested32_fixture_unchanged():
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_golden
    with open(os.path.join(HERE, "golden", "nested32_oracle.json")) as f:
        ref = json.load(f)
    now = make_golden.compute()
    assert now["x_sum"] == ref["x_sum"]
    np.testing.assert_allclose(now["fcm_init"]["centres"], ref["fcm_init"]["centres"], rtol=1e-13)
    assert now["fcm_init"]["iters"] == ref["fcm_init"]["iters"]
    for a, b in zip(now["solves"], ref["solves"]):
        assert a["iters"] == b["iters"]
        np.testing.assert_allclose(a["centres"], b["centres"], rtol=1e-12)
        np.testing.assert_allclose(a["J"], b["J"], rtol=1e-12)
        np.testing.assert_allclose(a["U_col_sums"], b["U_col_sums"], rtol=1e-12)
        assert a["label_counts"] == b["label_counts"]
