"""The Python binding checks every array's shape and layout against the
handle before a pointer reaches the C library (which reads as many doubles
as the shapes imply).  No device is needed: the checks fail before any
library call."""
import ctypes

import numpy as np
import pytest

from paper_2509_02840_amd import bdu


def _handle(m, n):
    h = bdu.Handle.__new__(bdu.Handle)
    h._h = ctypes.c_void_p()
    h.m, h.n = m, n
    return h


def _f(shape):
    return np.zeros(shape, order="F")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    bdu.lib()


def test_create_rejects_mismatched_factors():
    with pytest.raises(ValueError, match="Q"):
        bdu.Handle(_f((5, 4)), np.zeros(4), np.zeros(3), _f((4, 4)))
    with pytest.raises(ValueError, match="d"):
        bdu.Handle(_f((5, 5)), np.zeros(5), np.zeros(3), _f((4, 4)))
    with pytest.raises(ValueError, match="e"):
        bdu.Handle(_f((5, 5)), np.zeros(4), np.zeros(4), _f((4, 4)))
    with pytest.raises(ValueError, match="column-major"):
        bdu.Handle(np.zeros((5, 5)) + np.arange(5.0), np.zeros(4), np.zeros(3), _f((4, 4)))


def test_update_rejects_wrong_rows_and_ranks():
    h = _handle(6, 4)
    with pytest.raises(ValueError, match="B"):
        h.update(np.zeros(5), np.zeros(4))
    with pytest.raises(ValueError, match="C"):
        h.update(np.zeros(6), np.zeros(5))
    with pytest.raises(ValueError, match="columns"):
        h.update(_f((6, 2)), _f((4, 3)))
    with pytest.raises(ValueError, match="u"):
        h.update_projected(np.zeros(4), np.zeros(4))
    with pytest.raises(ValueError, match="b"):
        h.update_householder(np.zeros(7), np.zeros(4))
    with pytest.raises(ValueError, match="c"):
        h.project(np.zeros(6), np.zeros(3))
    with pytest.raises(ValueError, match="P"):
        h.read_into(P=_f((3, 3)))


def test_update_rejects_strided_views():
    h = _handle(6, 4)
    B = np.zeros((6, 4), order="F")[:, ::2]  # columns two apart: not packed
    with pytest.raises(ValueError, match="packed"):
        h.update(B, _f((4, 2)))
    with pytest.raises(ValueError, match="packed"):
        h.update(np.zeros(12)[::2], np.zeros(4))


def test_batched_calls_check_each_member():
    hs = [_handle(6, 4), _handle(9, 9)]
    with pytest.raises(ValueError, match="B"):
        bdu.update_batched(hs, [np.zeros(6), np.zeros(8)], [np.zeros(4), np.zeros(9)])
    with pytest.raises(ValueError, match="one B"):
        bdu.update_batched(hs, [np.zeros(6)], [np.zeros(4)])
    b = bdu.Batch.__new__(bdu.Batch)
    b._b = ctypes.c_void_p()
    b.handles = hs
    with pytest.raises(ValueError, match="both"):
        b.update([np.zeros(6), None], [np.zeros(4), np.zeros(9)])
    with pytest.raises(ValueError, match="exceeds"):
        b.update([np.zeros(6), None], [np.zeros(4), None], ranks=[1, 1])


def test_server_and_tracker_inputs():
    s = bdu.Server.__new__(bdu.Server)
    s._s = ctypes.c_void_p()
    s.shapes = {3: (6, 4)}
    with pytest.raises(ValueError, match="unknown"):
        s.submit(4, np.zeros(6), np.zeros(4))
    with pytest.raises(ValueError, match="C"):
        s.submit(3, np.zeros(6), np.zeros(6))
    with pytest.raises(ValueError, match="V"):
        bdu.Tracker(_f((8, 3)), np.zeros(3), np.zeros(2), _f((5, 2)))
    t = bdu.Tracker.__new__(bdu.Tracker)
    t._h = ctypes.c_void_p()
    t.m, t.n, t.r = 8, 5, 3
    with pytest.raises(ValueError, match="b"):
        t.update(np.zeros(5), np.zeros(5))
