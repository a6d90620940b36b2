"""Loaders of the paper's input formats (Aldebaran .aut files and the
EXP.OPEN par syntax of Fig. 1), checked against the worked example of Sec. 3
through the oracle."""
import os

import numpy as np
import pytest

import oracle
from paper_1801_05857_amd import models

from conftest import GOLDEN

FIG1 = os.path.join(GOLDEN, "fig1")


def _fig1():
    files = {n: open(os.path.join(FIG1, n)).read() for n in ("producer.aut", "consumer.aut")}
    return models.parse_par(open(os.path.join(FIG1, "network.exp")).read(), files)


def test_fig1_files_give_8_states_24_transitions():
    net = _fig1()
    assert net.n_states.tolist() == [2, 2, 2]
    assert net.rules.shape == (2, 3)
    r = oracle.explore(net)
    assert (r.n_states, r.n_transitions) == (8, 24)


def test_vector_semantics_by_position():
    net = _fig1()
    send, rec = net.labels.index("send"), net.labels.index("rec")
    assert net.rules.tolist() == [[send, rec, -1], [send, -1, rec]]


def test_aut_round_trip():
    text = models.write_aut(3, 1, [(0, "a", 1), (1, "b b", 2), (2, "i", 0)])
    lts = models.parse_aut(text)
    assert (lts.n_states, lts.initial) == (3, 1)
    assert lts.trans == [(0, "a", 1), (1, "b b", 2), (2, "i", 0)]


@pytest.mark.parametrize("bad", [
    "des (0, 1, 2)\n(0, \"a\", 5)\n",          # target out of range
    "des (0, 2, 2)\n(0, \"a\", 1)\n",          # count mismatch
    "des 0 1 2\n",                              # header
    "des (3, 0, 2)\n",                          # initial out of range
])
def test_aut_rejects_malformed(bad):
    with pytest.raises(ValueError):
        models.parse_aut(bad)


def test_par_rejects_malformed():
    aut = models.write_aut(1, 0, [])
    with pytest.raises(ValueError):
        models.parse_par('par using a * b -> c in "x.aut" end par', {"x.aut": aut})
    with pytest.raises(ValueError):
        models.parse_par('par using _ -> c in "x.aut" end par', {"x.aut": aut})
    with pytest.raises(ValueError):
        models.parse_par('par using a -> c in "y.aut" end par', {"x.aut": aut})
