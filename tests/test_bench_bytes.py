"""The benchmark's algorithmic byte counts (the numerator of its roofline fraction), checked against
the per-unit figures of the path written out by hand for the squeeze workload's block: a 10^3-hex
block of 1331 vertices and 6000 tets with 219 contacts, K = 20 local-global iterations.

Per local-global iteration: projection and assembly move 56 B per tet and 36 B per vertex; the
global apply 8 B per nonzero of a triangular factor's worth of the inverse (n (n + 1) / 2 nonzeros)
and 36 B per vertex; each Newton iteration of the contact solve 108 B per contact.  Per step: detection 24 B per vertex
and 64 B per contact, finalisation 48 B per vertex."""
import importlib.util
import os

from paper_2604_17513_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_path_bytes_of_one_squeeze_block():
    B = _bench()
    env = scenes.squeeze_blocks(1, seed=0).envs[0]
    assert env.n_vertices == 1331 and env.n_elements == 6000
    # one local-global iteration: projection + assembly 383,916 B, global apply 7,139,484 B
    one_lg = 383_916 + 7_139_484
    # the step: detection 31,944 + 14,016 B, 20 iterations, 11 Newton iterations of 23,652 B,
    # finalisation 63,888 B
    want = 31_944 + 14_016 + 20 * one_lg + 11 * 23_652 + 63_888
    assert want == 150_838_020
    assert B.path_bytes([env], [219], 20, [11.0]) == want
    # bytes add over envs and scale with the Newton count
    two = B.path_bytes([env, env], [219, 219], 20, [11.0, 12.0])
    assert two == 2 * want + 23_652


def test_overhead_and_apply_bytes():
    B = _bench()
    env = scenes.squeeze_blocks(1, seed=0).envs[0]
    # slot forces written and read back plus incidence slots (112 B per tet) and the position
    # update's read of the contact rows of the inverse (4 B per vertex per contact), per iteration
    assert B.overhead_bytes([env], [219], 20) == 20 * (672_000 + 1_165_956)
    # one batched apply launch as stored: the full n x n FP32 inverse and x, y, z in and out
    assert B.apply_bytes_per_launch([1331]) == 7_086_244 + 31_944
