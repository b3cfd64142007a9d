"""The event and gap pins have power: each rejects a copy of the oracle with
one rule broken the way a plausible mistake would break it.

Every case compiles a modified copy of the oracle source into a temporary
directory (CPU only) and runs one check of test_oracle_events.py against it;
the check must fail.  A case whose target text is no longer in the source
fails too, so a rewrite of the oracle cannot silently disarm it.
"""
import pytest

import oracle
from test_oracle_events import (check_dissolution, check_gap, check_normal_refresh,
                                check_precipitation)
from test_oracle_adjoint import check_gap_adjoint

MUTANTS = [
    # dissolution: the new cell's C as the sum, not the mean, of its fluid neighbours
    ("sum instead of mean", "double Cs = csum / nf, rs = rsum / nf;",
     "double Cs = csum, rs = rsum / nf;", check_dissolution),
    # dissolution: the deficit split evenly instead of by rate constant
    ("unweighted deficit split", "wt[nn] = o->kr[y];\n                wsum += o->kr[y];",
     "wt[nn] = 1.0;\n                wsum += 1.0;", check_dissolution),
    # dissolution: the deficit added instead of removed
    ("deficit sign", "o->phi[nb[k]] -= need *", "o->phi[nb[k]] += need *", check_dissolution),
    # precipitation: the local concentration not turned into phi
    ("concentration not converted", "o->phi[n] += vm * Cx;", "(void)Cx;", check_precipitation),
    # precipitation: the excess not passed on
    ("excess kept", "o->phi[nb[k]] += excess / nn;", "o->phi[nb[k]] += 0.0 * excess;",
     check_precipitation),
    # precipitation: every share the whole excess
    ("excess not split", "o->phi[nb[k]] += excess / nn;", "o->phi[nb[k]] += excess;",
     check_precipitation),
    # normals refreshed within one site only
    ("refresh radius", "int r = 2, zr = o->p.dim == 3 ? 2 : 0;",
     "int r = 1, zr = o->p.dim == 3 ? 1 : 0;", check_normal_refresh),
    # one-node gap: the post-collision fallback keeps gamma k
    ("gap keeps gamma", "if (p->mechanics == ORC_MECH_PRE) k = k / o->gamma;", "",
     lambda lib: check_gap(9, 0, lib)),
    ("gap keeps gamma (3D)", "if (p->mechanics == ORC_MECH_PRE) k = k / o->gamma;", "",
     lambda lib: check_gap(19, 0, lib)),
    # the adjoint's one-node gap: the derivative without the 1/gamma
    ("adjoint gap keeps gamma",
     "if (!pulled && p->mechanics == ORC_MECH_PRE) { k = k / o->gamma; dk = dk / o->gamma; }",
     "if (!pulled && p->mechanics == ORC_MECH_PRE) { k = k / o->gamma; }", check_gap_adjoint),
]


@pytest.mark.parametrize("name,old,new,check", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_rejects_planted_mistake(tmp_path, name, old, new, check):
    with open(oracle.SRC) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"mutation target of '{name}' not found once in the oracle"
    lib = oracle.load_variant(src.replace(old, new), str(tmp_path))
    with pytest.raises(AssertionError):
        check(lib)


def test_unmodified_copy_passes(tmp_path):
    """The same compile-and-load route with the source unchanged passes every check."""
    with open(oracle.SRC) as fh:
        lib = oracle.load_variant(fh.read(), str(tmp_path))
    check_dissolution(lib)
    check_precipitation(lib)
    check_normal_refresh(lib)
    check_gap(9, 0, lib)
    check_gap_adjoint(lib)
