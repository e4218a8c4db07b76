"""The flatten pass of the voxel labelling under randomized schedules (CPU
model in tests/vol_flatten_model.py): the shipped read-only walk gives every
voxel its root in every schedule tried; the first version, which compressed
the paths it walked, can overwrite a root already written by its owner with
a stale non-root ancestor -- the cause of the non-minimal volume labels seen
on the GPU before the fix."""
import numpy as np

from tests import vol_flatten_model as M


def forests(rng):
    yield [0, 0, 1, 2, 3, 4, 5, 6]          # one long chain
    yield [0, 0, 0, 1, 1, 2, 2, 3, 3, 4]    # a binary tree
    for _ in range(20):
        n = int(rng.integers(2, 40))
        yield [0] + [int(rng.integers(0, v + 1)) for v in range(1, n)]


def test_read_only_walk_always_gives_roots():
    rng = np.random.default_rng(1)
    for f in forests(rng):
        want = M.roots(f)
        for s in range(30):
            assert M.flatten(f, "read", s) == want


def test_compressing_walk_can_leave_a_non_root():
    chain = [0, 0, 1, 2, 3, 4, 5, 6]
    bad = [s for s in range(300) if M.flatten(chain, "compress", s) != M.roots(chain)]
    assert bad, "expected a schedule in which compression overwrites a finished entry"
