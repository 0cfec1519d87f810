"""CPU tests of the LAMMPS-format parameter-file parser of libtersoff.so
(host code only; no device needed).  The files are written here from the
tables of the workload module in the documented 17-word entry layout."""
import numpy as np
import pytest

from paper_1710_00882_amd import workloads as W

ORDER = ("m", "gamma", "lambda3", "c", "d", "h", "eta", "beta", "lambda2", "B", "R", "D", "lambda1", "A")
FIELD = {name: k for k, name in enumerate(W.PARAM_FIELDS)}


def to_file(table, elements, split_lines=False, comments=True):
    nt = len(elements)
    table = np.asarray(table).reshape(-1, 14)
    out = ["# element1 element2 element3 m gamma lambda3 c d costheta0 n beta lambda2 B R D lambda1 A"] if comments else []
    for ti in range(nt):
        for tj in range(nt):
            for tk in range(nt):
                row = table[(ti * nt + tj) * nt + tk]
                vals = [repr(float(row[FIELD[f]])) for f in ORDER]
                words = [elements[ti], elements[tj], elements[tk]] + vals
                if split_lines:
                    out.append(" ".join(words[:9]))
                    out.append("   " + " ".join(words[9:]) + ("  # continued" if comments else ""))
                else:
                    out.append(" ".join(words))
    return "\n".join(out) + "\n"


@pytest.fixture(scope="module")
def parse():
    from paper_1710_00882_amd import _lib
    import os
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libtersoff.so not built")
    return _lib.parse_params


def test_field_order_matches_workloads():
    assert set(ORDER) == set(W.PARAM_FIELDS)


def test_round_trip_one_species(parse):
    t = W.si_table()
    got = parse(to_file(t, ["Si"]), ["Si"])
    assert np.array_equal(got, t.reshape(-1, 14))


@pytest.mark.parametrize("split", [False, True])
def test_round_trip_two_species(parse, split):
    t = W.two_species_table()
    got = parse(to_file(t, ["Si", "X"], split_lines=split), ["Si", "X"])
    assert np.array_equal(got, t.reshape(-1, 14))


def test_element_order_defines_types(parse):
    t = W.two_species_table().reshape(8, 14)
    got = parse(to_file(t, ["Si", "X"]), ["X", "Si"])   # type 0 is now X
    for ti in range(2):
        for tj in range(2):
            for tk in range(2):
                src = ((1 - ti) * 2 + (1 - tj)) * 2 + (1 - tk)
                assert np.array_equal(got[(ti * 2 + tj) * 2 + tk], t[src])


def test_unrequested_elements_are_skipped(parse):
    t = W.two_species_table()
    got = parse(to_file(t, ["Si", "X"]), ["Si"])
    assert np.array_equal(got[0], t.reshape(-1, 14)[0])


def test_errors(parse):
    from paper_1710_00882_amd import TersoffError
    t = W.si_table()
    good = to_file(t, ["Si"], comments=False)
    with pytest.raises(TersoffError):
        parse(good + good, ["Si"])                          # triplet twice
    with pytest.raises(TersoffError):
        parse(good, ["Si", "C"])                             # entries with C missing
    with pytest.raises(TersoffError):
        parse(good.replace(repr(float(t.reshape(-1, 14)[0][FIELD["A"]])), "1.0.0"), ["Si"])   # malformed number
    with pytest.raises(TersoffError):
        parse(good + " Si", ["Si"])                          # word count not a multiple of 17
    with pytest.raises(TersoffError):
        parse(good, [])
