"""The C-ABI library loads, exports every function include/pic.h declares, and rejects bad
arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest
import torch

import paper_2208_02382_amd as pic
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pic.h")).read()
    return sorted(set(re.findall(r"^(?:pic_status|size_t|const char\*)\s+(pic_\w+)\(", text,
                                 re.M)))


def test_header_symbols_are_exported():
    names = _declared()
    assert len(names) == 28
    lib = ctypes.CDLL(pic.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def _desc(**kw):
    c = workloads.SMALL
    d = dict(n=c.n, qm_qeeV=c.qm_qeeV, charge_C=c.charge_C, kin_energy_MeV=c.kin_energy_MeV,
             mass_MeV=c.mass_MeV, shape=c.shape, nodes=c.nodes)
    d.update(kw)
    return pic.make_desc(**d)


def test_workspace_bytes_validates_the_description():
    assert pic.workspace_bytes(_desc()) > 0
    assert pic.workspace_bytes(_desc(nodes=(48, 32, 96))) > 0      # 96 and 192 = 2^a 3^b
    assert pic.workspace_bytes(_desc(shape=3)) == 0
    assert pic.workspace_bytes(_desc(nodes=(3, 32, 32))) == 0
    assert pic.workspace_bytes(_desc(nodes=(7, 32, 32))) == 0       # 14 = 2 * 7
    assert "2^a 3^b" in pic.last_error()
    assert pic.workspace_bytes(_desc(nodes=(320, 32, 32))) == 0     # 640 > 512
    assert pic.workspace_bytes(_desc(n=0)) == 0
    assert pic.workspace_bytes(_desc(kin_energy_MeV=-1.0)) == 0


def test_tuning_fields_are_validated():
    base = pic.workspace_bytes(_desc())
    assert pic.workspace_bytes(_desc(tuning={"tile": (8, 8, 8), "chunk": 2048, "blocks": 512})) > 0
    # smaller chunks need a longer work list
    assert pic.workspace_bytes(_desc(nodes=(64, 64, 64), n=10**6, tuning={"chunk": 256})) > \
        pic.workspace_bytes(_desc(nodes=(64, 64, 64), n=10**6))
    assert pic.workspace_bytes(_desc(tuning={"tile": (1, 1, 1)})) == 0     # 32^3 tiles > 4096
    assert "4096" in pic.last_error()
    assert pic.workspace_bytes(_desc(tuning={"tile": (33, 4, 4)})) == 0    # tile > n
    assert pic.workspace_bytes(_desc(tuning={"tile": (32, 32, 8)})) > 0    # 78 KB window
    assert pic.workspace_bytes(_desc(tuning={"tile": (32, 32, 32)})) == 0  # window > 160 KB
    assert "LDS" in pic.last_error()
    assert pic.workspace_bytes(_desc(tuning={"threads": 1024})) == base
    assert pic.workspace_bytes(_desc(tuning={"deposit_threads": 128})) == base
    for bad in (32, 100, 2048, -64):
        assert pic.workspace_bytes(_desc(tuning={"threads": bad})) == 0
        assert pic.workspace_bytes(_desc(tuning={"deposit_threads": bad})) == 0
    assert pic.workspace_bytes(_desc(tuning={"tile": (-1, 0, 0)})) == 0
    assert pic.workspace_bytes(_desc(tuning={"chunk": 100})) == 0
    assert pic.workspace_bytes(_desc(tuning={"blocks": 70000})) == 0
    assert pic.workspace_bytes(_desc()) == base


def _lat_ptrs(*lats):
    arrs = [pic._lattice(l) for l in lats]
    ptrs = (ctypes.POINTER(pic.Element) * len(arrs))(
        *[ctypes.cast(a, ctypes.POINTER(pic.Element)) for a in arrs])
    return arrs, ptrs, (ctypes.c_int * len(arrs))(*[len(l) for l in lats])


def test_batch_arguments_are_validated_without_a_device():
    lib = pic._lib
    keep, ptrs, n_el = _lat_ptrs(((1.0, 0.5), (-1.0, 0.5)), ((1.0, 0.5),))
    n_el[1] = 0
    assert lib.pic_batch_workspace_bytes(2, ptrs, n_el) == 0             # an empty lattice
    n_el[1] = 1
    thin = lib.pic_batch_workspace_bytes(2, ptrs, n_el)
    assert thin > 0
    assert lib.pic_batch_workspace_bytes(0, ptrs, n_el) == 0
    # thick elements expand into slices: a larger table
    keep2, ptrs2, n_el2 = _lat_ptrs(((1.0, 0.5), (-1.0, 0.5)), ((2, 1.0, 1.0, 400),))
    assert lib.pic_batch_workspace_bytes(2, ptrs2, n_el2) > thin
    out = ctypes.c_void_p()
    assert lib.pic_batch_create(None, 2, None, n_el, 0, None, 0, None, ctypes.byref(out)) \
        == pic.PIC_EINVAL
    assert lib.pic_track_batch(None, 3, None) == pic.PIC_EINVAL


def test_lattice_elements_are_validated():
    lib = pic._lib
    for bad in (((5, 1.0, 1.0, 1),),           # unknown kind
                ((2, 1.0, 1.0, 0),),           # no slices
                ((1, 0.0, -0.5, 2),),          # negative length
                ((2, float("nan"), 1.0, 3),)):
        keep, ptrs, n_el = _lat_ptrs(bad)
        assert lib.pic_batch_workspace_bytes(1, ptrs, n_el) == 0
    keep, ptrs, n_el = _lat_ptrs(((1, 0.0, 0.25, 25), (2, 1.0, 1.0, 25)))
    assert lib.pic_batch_workspace_bytes(1, ptrs, n_el) > 0


def test_create_rejects_bad_arguments_without_touching_a_device():
    lib = pic._lib
    d = _desc()
    nbytes = pic.workspace_bytes(d)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x10000)
    assert lib.pic_beam_create(ctypes.byref(d), None, fake, nbytes, None, ctypes.byref(h)) == pic.PIC_EINVAL
    assert lib.pic_beam_create(ctypes.byref(d), fake, ctypes.c_void_p(0x10008), nbytes, None,
                               ctypes.byref(h)) == pic.PIC_EINVAL   # misaligned workspace
    assert lib.pic_beam_create(ctypes.byref(d), fake, fake, nbytes - 1, None,
                               ctypes.byref(h)) == pic.PIC_ENOMEM
    bad = _desc(nodes=(10, 32, 32))   # 20 = 2^2 * 5
    assert lib.pic_beam_create(ctypes.byref(bad), fake, fake, nbytes, None,
                               ctypes.byref(h)) == pic.PIC_EUNSUPPORTED
    assert lib.pic_beam_create(None, fake, fake, nbytes, None, ctypes.byref(h)) == pic.PIC_EINVAL
    assert lib.pic_track_n_steps(None, None, 0, 0, None) == pic.PIC_EINVAL
    assert lib.pic_deposit(None, None, None) == pic.PIC_EINVAL
    assert lib.pic_moments(None, None, None, None) == pic.PIC_EINVAL
    assert lib.pic_objective(None, None, None) == pic.PIC_EINVAL
    assert lib.pic_beam_destroy(None) == pic.PIC_OK


@pytest.mark.skipif(torch.cuda.device_count() > 0, reason="a device is present")
def test_create_reports_no_device():
    d = _desc()
    nbytes = pic.workspace_bytes(d)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x10000)
    st = pic._lib.pic_beam_create(ctypes.byref(d), fake, fake, nbytes, None, ctypes.byref(h))
    assert st == pic.PIC_ENODEV
    assert h.value is None


def test_sigma_from_params_matches_the_oracle():
    # host-only entry point: the Listing 1 parameters and a correlated longitudinal plane
    from oracle import pic as opic
    import numpy as np
    for args in ((3.9984884770e-5, 3.9984884770e-5, 1.0e-3, 2.6623538760e-5, 2.6623538760e-5,
                  2.0e-3, -0.846574929020762, 0.846574929020762, 0.0),
                 (1e-3, 2e-3, 3e-3, 4e-4, 5e-4, 6e-4, 0.3, -0.5, 0.7)):
        got = np.array(pic.sigma_from_params(*args))
        ref = opic.sigma_from_params(*args)
        assert np.allclose(got, ref, rtol=1e-15, atol=0)
    for bad in ((0.0, 1, 1, 1, 1, 1, 0, 0, 0), (1, 1, 1, 1, 1, 1, 1.0, 0, 0),
                (1, 1, float("nan"), 1, 1, 1, 0, 0, 0)):
        with pytest.raises(pic.PicError):
            pic.sigma_from_params(*bad)


def test_direct_field_flag_is_validated():
    base = pic.workspace_bytes(_desc())
    # the field kernels' corners, octant arrays, spectra and a second work array
    assert pic.workspace_bytes(_desc(direct_field=True)) > base
    d = _desc()
    d.direct_field = 2
    assert pic.workspace_bytes(d) == 0
    assert "direct_field" in pic.last_error()
