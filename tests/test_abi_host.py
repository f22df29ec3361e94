"""Host-side checks of libnat_bem.so that need no GPU: it loads, exports every
entry point include/nat_bem.h declares, validates meshes, and builds the
FP64 area table bit for bit like the oracle (the precondition for
bit-exact sample triangle indices)."""
import re
from pathlib import Path

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O
from paper_2506_06190_amd import nat

HEADERS = sorted((Path(__file__).resolve().parents[1] / "include").glob("*.h"))


def declared_functions():
    names = []
    for h in HEADERS:
        names += re.findall(r"^[A-Za-z_][\w \*]*?\b(nat_\w+)\s*\(", h.read_text(), re.M)
    return names


def test_library_exports_every_declared_symbol():
    L = nat.lib()
    names = declared_functions()
    assert len(HEADERS) == 3 and len(names) >= 34
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps each of them under the same name
    assert set(names) <= set(nat._SIGS)


def test_neural_field_calls_validate_before_device_work():
    """The neural-field calls refuse missing handles and bad sizes on the
    host (no device is touched)."""
    import ctypes as C
    L = nat.lib()
    h = C.c_void_p()
    assert L.nat_nf_create(None, 0, 1, 1.5, 3.0, 0, C.byref(h)) == nat.NAT_E_INVALID
    assert "context is NULL" in nat.last_error()
    assert L.nat_nf_create(None, 0, 1, 1.5, 3.0, 0, None) == nat.NAT_E_INVALID
    assert L.nat_nf_info(None, None, None) == nat.NAT_E_INVALID
    assert L.nat_nf_infer(None, None, 4, None, None) == nat.NAT_E_INVALID
    assert L.nat_nf_train_step(None, None, None, 4, 0, 1, None, None) == nat.NAT_E_INVALID
    assert L.nat_nf_get_params(None, None, 0) == nat.NAT_E_INVALID
    L.nat_nf_destroy(None)


def test_status_strings_and_defaults():
    assert nat.status_str(nat.NAT_OK) == "NAT_OK"
    assert nat.status_str(nat.NAT_E_BUDGET) == "NAT_E_BUDGET"
    assert nat.status_str(nat.NAT_E_CANCELLED) == "NAT_E_CANCELLED"
    so = nat.nat_server_opts_default()
    assert so.n_slots == 4 and so.max_batch == 64 and so.hbm_budget == 16 << 30
    assert so.mc.gmres_tol == 1e-6 and so.dense_tol == 1e-6 and so.dense_burton_miller == 1
    o = nat.nat_mc_opts_default()
    assert o.gmres_tol == 1e-6 and o.gmres_max_iter == 200     # Section 6.1 solver settings
    assert o.eps_scale == 1.0 and o.precision == nat.NAT_PREC_FP32 and o.flags == 0


@pytest.mark.parametrize("maker", [
    lambda: W.icosphere(3, 1.0)[:2],
    lambda: W.noisy_ellipsoid(3, subdiv=3)[:2],
    lambda: W.cubesphere_ellipsoid(5, 3000)[:2],
])
def test_geometry_bitwise_equal_to_oracle(maker):
    v, f = maker()
    a1, n1, c1 = nat.nat_mesh_geometry(v, f)
    a2, n2, c2 = O.geometry(v, f)
    assert np.array_equal(a1, a2) and np.array_equal(n1, n2) and np.array_equal(c1, c2)


def test_mesh_validation_rejects_bad_meshes():
    v, f, _ = W.icosphere(1, 1.0)
    assert nat.nat_mesh_validate(v, f)[0] == nat.NAT_OK
    bad = {
        "open": (v, f[1:]),
        "one triangle flipped": (v, np.concatenate([f[:1, [0, 2, 1]], f[1:]])),
        "inward": (v, f[:, [0, 2, 1]]),
        "index out of range": (v, np.where(f == 3, len(v), f)),
        "repeated vertex": (v, np.concatenate([f[:1, [0, 0, 1]], f[1:]])),
    }
    for name, (vv, ff) in bad.items():
        st, msg = nat.nat_mesh_validate(vv, ff)
        assert st == nat.NAT_E_INVALID, name
        assert msg, name
    vn = v.copy()
    vn[5, 1] = np.nan
    assert nat.nat_mesh_validate(vn, f)[0] == nat.NAT_E_INVALID
    # a zero-area triangle: collapse one vertex onto another's position
    vz = v.copy()
    t0 = f[0]
    vz[t0[2]] = vz[t0[1]]
    st, msg = nat.nat_mesh_validate(vz, f)
    assert st == nat.NAT_E_INVALID and "zero area" in msg


def test_batch_job_layout_must_match_the_batch():
    """A job whose Neumann data was shaped for one layout cannot enter a batch
    run with the other (the C job record has no layout of its own, so the
    library would read v_n with the batch's layout)."""
    job = nat.McJob.__new__(nat.McJob)
    job.layout = nat.NAT_NEUMANN_PER_VERTEX
    with pytest.raises(ValueError, match="layout"):
        job.record(nat.NAT_NEUMANN_PER_TRIANGLE)
    job.layout = nat.NAT_NEUMANN_PER_TRIANGLE
    with pytest.raises(ValueError, match="layout"):
        job.record(nat.NAT_NEUMANN_PER_VERTEX)


def test_scene_of_several_bodies_validated_per_body():
    """A mesh of several closed bodies is accepted when every body is
    oriented outward; turning any one body inside out is refused, naming it
    (the total volume of the scene would still be positive)."""
    sc = W.scene_speaker_torus(0.03)
    assert nat.nat_mesh_validate(sc.vertices, sc.tris) == (nat.NAT_OK, "")
    for b in (0, 1):
        f = sc.tris.copy()
        f[sc.body == b] = f[sc.body == b][:, [0, 2, 1]]
        st, msg = nat.nat_mesh_validate(sc.vertices, f)
        assert st == nat.NAT_E_INVALID and f"body {b} of 2" in msg
    # the geometry of a scene equals the oracle's bit for bit, as for one body
    area, nrm, cdf = nat.nat_mesh_geometry(sc.vertices, sc.tris)
    ao, no, co = O.geometry(sc.vertices, sc.tris)
    assert np.array_equal(area, ao) and np.array_equal(nrm, no) and np.array_equal(cdf, co)
