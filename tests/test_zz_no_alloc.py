"""mb_run_static: the run entry point that allocates nothing (group tables in the
library's static device scratch) gives the same records as mb_run."""
import numpy as np
import pytest

import paper_2005_05412_amd as mb
import workloads as W

pytestmark = pytest.mark.gpu


def _records(prob, static, chunks=None, **shape):
    s = mb.Solver(prob, **shape)
    run = s.run_static if static else s.run
    for c in chunks or []:
        run(c)
    run()
    out = s.records()
    s.close()
    return out


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("shape", [dict(precision=32, variant="blocked", block=256, depth=32),
                                   dict(precision=64, variant="blocked", block=128, depth=48),
                                   dict(precision=64, variant="plain")],
                         ids=["persistent-fp32", "chunks-fp64", "plain-fp64"])
def test_static_run_equals_run_twice_in_a_row(shape):
    """A large problem, then a smaller one right after it (the scratch holds the first
    run's tables), each equal bit for bit to mb_run's records."""
    big = W.random_small(51, N=3, nx=2000, n_steps=300, refl=(0.0, 0.0), rec_interval=10)
    small = W.random_small(52, N=2, nx=150, n_steps=200, refl=(1.0, 0.0), rec_interval=10)
    if shape.get("depth") == 32:      # this shape's solves run as persistent launches
        s = mb.Solver(big, **shape)
        assert s.persistent()
        s.close()
    for prob in (big, small):
        _same(_records(prob, True, **shape), _records(prob, False, **shape))
    # one solve in pieces: the flags and step bookkeeping carry over between calls
    _same(_records(big, True, chunks=[7, 100], **shape), _records(big, False, **shape))


def test_static_run_rejects_tables_beyond_the_scratch():
    """A grid of more tiles than the scratch can describe is refused before any launch."""
    nx = 24 * 60000  # 64-cell tiles of 24 owned cells: 60000 tiles, 1.2 MB of tables
    prob = W.random_small(53, N=0, nx=nx, n_steps=5, refl=(0.0, 0.0), full_records=False)
    s = mb.Solver(prob, precision=32, variant="blocked", block=64, depth=20)
    with pytest.raises(mb.MBError) as ex:
        s.run_static()
    assert ex.value.code == -5 and "static scratch" in str(ex.value)
    s.run()          # the ordinary entry point still runs it
    s.close()
