"""The oracle against hand-derived fixtures (tests/golden/, each citing the
definition it was worked out from)."""
import numpy as np
import pytest

import oracle
from tests import golden_io


@pytest.mark.parametrize("path", golden_io.all_fixtures(), ids=lambda p: p.split("/")[-1])
def test_fixture(path):
    fx = golden_io.load(path)
    B = fx["blocks"]
    op = fx["op"]
    if op == "formula":
        outs = oracle.run("\n".join(B["formula"]), golden_io.image(fx))
        assert np.array_equal(outs[0], golden_io.mask(B["expect"]))
    elif op == "ccl":
        a = golden_io.mask(B["a"])
        lab = oracle.ccl(a)
        letters = np.array([list(r) for r in B["expect"]])
        w = a.shape[1]
        for ch in set(letters.reshape(-1)) - {"."}:
            ys, xs = np.nonzero(letters == ch)
            assert set(lab[ys, xs].tolist()) == {int(min(ys * w + xs))}
        assert np.all(lab[letters == "."] == -1)
    else:
        a = golden_io.mask(B["a"])
        fn = getattr(oracle, op)
        got = fn(a, golden_io.mask(B["b"])) if "b" in B else fn(a)
        assert np.array_equal(got, golden_io.mask(B["expect"])), got
