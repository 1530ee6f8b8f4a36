"""Values the paper prints, kept as text fixtures under tests/golden/ (each
with its citation), against the code that uses them.

tab_mg.txt: the multigrid parameters of tab. mg (Section 3.4).  The package's
table and every V-cycle default (library binding and oracle) must be the
paper's, so that a run without explicit parameters is the paper's method."""
import inspect
import os

from oracle import cavity as CV
from oracle import sweep as SW

HERE = os.path.dirname(__file__)


def _tab_mg():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "tab_mg.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        dim, order, coarsest, pre, post = (int(x) for x in line.split())
        rows[(dim, order)] = (coarsest, pre, post)
    return rows


def _defaults(fn):
    sig = inspect.signature(fn)
    return tuple(sig.parameters[k].default for k in ("coarsest", "nu1", "nu2"))


def test_fixture_holds_the_four_rows_of_the_table():
    rows = _tab_mg()
    assert sorted(rows) == [(1, 1), (1, 2), (2, 1), (2, 2)]
    # more smoothing for the second-order schemes, one post-smoothing step throughout
    assert all(rows[(d, 2)][1] > rows[(d, 1)][1] for d in (1, 2))
    assert all(r[2] == 1 for r in rows.values())


def test_package_table_is_the_papers():
    import paper_2409_01910_amd as bz

    assert bz.MG_PARAMS == _tab_mg()
    for (dim, order), (c, n1, n2) in _tab_mg().items():
        assert bz.mg_params(dim, order) == {"coarsest": c, "nu1": n1, "nu2": n2}


def test_vcycle_defaults_are_the_first_order_rows():
    import paper_2409_01910_amd as bz

    rows = _tab_mg()
    assert _defaults(bz.Slab.vcycle) == rows[(1, 1)]
    assert _defaults(bz.Slab.capture_vcycles) == rows[(1, 1)]
    assert _defaults(bz.Cavity.vcycle) == rows[(2, 1)]
    assert _defaults(SW.solve_mg) == rows[(1, 1)]
    assert _defaults(CV.mg_iteration) == rows[(2, 1)]
