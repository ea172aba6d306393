import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU")
    config.addinivalue_line("markers", "slow: long CPU physics pin")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden_rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


class Golden:
    """Values the paper prints, read from the cited text fixtures."""

    def table2(self):
        """{name: (optimal, lower, upper)} of Table 2."""
        return {r[0]: tuple(float(v) for v in r[1:4])
                for r in _golden_rows("table2_relaxation_parameters.txt")}

    def table2_row(self):
        """Table 2 in the relaxation-row order of the library and the oracle:
        kappa_x1, kappa_x2, d_x1[nu], d_x2[nu], alpha_x1[nu], alpha_x2[nu]."""
        t = self.table2()
        names = ["kappa_x1", "kappa_x2"] + [
            "%s_%s_nu%d" % (q, x, nu) for q in ("d", "alpha")
            for x in ("x1", "x2") for nu in (1, 2)]
        return [t[n][0] for n in names]

    def stated(self):
        """{key: value} of the paper's stated setup and validation figures."""
        return {r[0]: float(r[1]) for r in _golden_rows("stated_results.txt")}


@pytest.fixture(scope="session")
def golden():
    return Golden()


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import solver
    solver.build()
    return solver
