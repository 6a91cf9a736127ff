"""The autotuner on the GPU: a single-mesh search and a mix search (the server's
table entry), their table entries and the cached second call.

The search is coordinate descent from the defaults over measured Rosenbrock
steps, so the chosen launch configuration is a timing outcome; what is fixed is
that it lies in the searched set, that it is no slower than the defaults it was
measured against, that a mix searches rows per thread only, and that the table
then answers lookups with it."""
import pytest

from helpers import Problem

pytestmark = pytest.mark.gpu

KNOBS = {"rows_per_thread": (1, 2, 4, 8), "ticks_per_graph": (32, 64, 128), "pcg_steps_per_launch": (1, 2),
         "grid_columns": (0, 1), "shared_ops": (0, 1)}


@pytest.fixture()
def pfc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06852_amd import pfc as lib
    lib.pfc_tune_clear()
    yield lib
    lib.pfc_tune_clear()


def _in_searched_set(e):
    for k, values in KNOBS.items():
        assert e[k] in values, (k, e[k])
    assert 0.0 < e["ms_per_step"] <= e["ms_default"]


def test_autotune_single_mesh_entry_and_cache(pfc):
    P = Problem(2, 64, seed=3)
    try:
        m = P.gpu_mesh()
        e = pfc.pfc_autotune(m, 0, 1, force=True)
        _in_searched_set(e)
        assert (e["dim"], e["n"], e["precision"], e["count"], e["from_cache"]) == (2, P.n, 0, 1, 0)
        # the defaults first, then rows per thread, column form, PCG form and graph length
        assert 2 <= e["candidates"] <= 10
        # the two-iteration form needs one row per thread
        assert e["pcg_steps_per_launch"] == 1 or e["rows_per_thread"] == 1
        again = pfc.pfc_autotune(m, 0, 1)
        assert again["from_cache"] == 1
        for k in KNOBS:
            assert again[k] == e[k], k
        look = pfc.pfc_tune_lookup(2, P.n, e["z"], 0, 1)
        assert look is not None and look["rows_per_thread"] == e["rows_per_thread"]
    finally:
        P.close()


def test_autotune_mix_entry(pfc):
    # a 2D grid of side 64 (whose instances keep the block form in a mix) and a 3D grid
    Ps = [Problem(2, 64, seed=4), Problem(3, 8, seed=5)]
    try:
        ms = [P.gpu_mesh() for P in Ps]
        e = pfc.pfc_autotune_mix(ms, 1, 4, force=True)
        _in_searched_set(e)
        assert (e["dim"], e["n"], e["z"], e["precision"], e["count"], e["from_cache"]) == (0, 0, 0, 1, 4, 0)
        # a mix searches the rows per thread alone (the defaults included)
        assert 1 <= e["candidates"] <= 4
        look = pfc.pfc_tune_lookup(0, 0, 0, 1, 4)
        assert look is not None and look["rows_per_thread"] == e["rows_per_thread"]
        assert pfc.pfc_tune_lookup(0, 0, 0, 1, 3) is None
    finally:
        for P in Ps:
            P.close()
