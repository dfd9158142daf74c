import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as o
    o.lib()
    return o


_codes = {}


def code_pair(name):
    """(spec, OracleCode) for a named instance, cached per session."""
    from lead_inputs import standard, custom_code
    from oracle.oracle import OracleCode
    if name not in _codes:
        if name in ("T", "M", "L"):
            spec = standard(name)
        elif name == "appendix":
            # rep[3,1] and the even-weight [3,2] code over (Z_2)^3, Delta = 3
            spec = custom_code("E2_3", 3, [1, 2, 4], [3, 6, 5], [0b111], [0b011, 0b110])
        elif name == "Z5":
            spec = custom_code("Z5", 2, [1, 4], [2, 3], [0b11], [0b11])
        elif name == "D3":
            spec = custom_code("D3", 2, [1, 2], [3, 4], [0b11], [0b11])
        elif name == "T_pairs":
            # [4,2] "pair" codes: every local variable sits in one check (a forest)
            t = standard("T")
            spec = custom_code("D6", 4, t.A, t.B, [0b0011, 0b1100], [0b0101, 0b1010])
        else:
            raise KeyError(name)
        _codes[name] = (spec, OracleCode.from_spec(spec))
    return _codes[name]
