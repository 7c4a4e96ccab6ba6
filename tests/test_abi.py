"""The C ABI without a GPU: the library is built, loads, exports every function that
include/dmts.h declares, and rejects bad arguments on the host before touching the
device."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_06562_amd import api, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "dmts.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:nnp|dmts)_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = api.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(api.EXPORTED)


def test_version_string():
    assert b"gfx950" in api.lib().dmts_version()


def test_model_create_rejects_wrong_blob_size():
    d = api.ModelDesc(kind=0, cutoff=3.5, n_rbf=16, width=64)
    w = np.zeros(10, dtype=np.float32)
    with pytest.raises(api.DmtsError) as e:
        api.Model(d, w)
    assert e.value.status == api.E_ARG
    assert "weights" in str(e.value)


def test_model_create_rejects_unsupported_shape():
    d = api.ModelDesc(kind=1, cutoff=5.2, n_rbf=16, width=128)
    with pytest.raises(api.DmtsError) as e:
        api.Model(d, synth.model_weights(synth.LARGE, 1))
    assert e.value.status == api.E_ARG


def test_nlist_create_rejects_bad_alignment():
    h = ctypes.c_void_p()
    assert api.lib().nnp_nlist_create(10, 100, 3, ctypes.byref(h)) == api.E_ARG
    assert api.lib().nnp_nlist_create(0, 100, 4, ctypes.byref(h)) == api.E_ARG


def test_state_create_rejects_bad_arguments():
    h = ctypes.c_void_p()
    m = np.ones(5)
    L = api.lib()
    sp = ctypes.c_void_p(16)   # never dereferenced: the call fails validation first
    assert L.dmts_state_create(0, 10.0, sp, m.ctypes.data_as(ctypes.c_void_p), 5, 1.0, 1, 8, 8,
                               ctypes.byref(h)) == api.E_ARG
    assert L.dmts_state_create(10, 10.0, sp, m.ctypes.data_as(ctypes.c_void_p), 5, 1.0, 0, 8, 8,
                               ctypes.byref(h)) == api.E_ARG
    bad = np.array([1.0, 0.0, 1.0, 1.0, 1.0])
    assert L.dmts_state_create(10, 10.0, sp, bad.ctypes.data_as(ctypes.c_void_p), 5, 1.0, 1, 8, 8,
                               ctypes.byref(h)) == api.E_ARG


def test_null_arguments_are_rejected():
    L = api.lib()
    assert L.nnp_energy_forces(None, None, None, None, 0, 0.0, None, 1, None, None, None,
                               None) == api.E_ARG
    assert L.dmts_step(None, None, None, None, None, 1, None, None) == api.E_ARG
    assert L.nnp_build_neighbors(None, None, 0, 0.0, None, 1, 3.5, None) == api.E_ARG
    assert b"null" in L.dmts_last_error()
