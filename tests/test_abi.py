"""The C ABI on the CPU: the library loads, exports every entry point that
include/prc.h declares, and its host-only calls (parameter setup,
validation, layout, sizes) behave as documented.  Nothing here launches a
kernel."""
import os
import re

import pytest

from paper_2208_03562_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(prc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_entry_point():
    L = capi.lib()
    names = declared_entry_points()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(capi.exported_names())


def base():
    p = capi.prc_params_default()
    p.nx, p.ny = 64, 32
    return p


def test_defaults_are_the_papers_rates():
    p = capi.prc_params_default()
    assert (p.omega_xi, p.omega_1, p.omega_3, p.omega_4) == (1.0, 1.0, 1.0, 1.0)
    assert p.corrections == capi.PRC_CORR_ALL and p.frame == capi.PRC_FRAME_CENTRAL


def test_omega_from_re_matches_oracle(O):
    for r, g, re_, U, ny in [(2.0, 1.0, 100, 0.05, 32), (2.0, 0.1, 1000, 0.05, 512),
                             (0.5, 0.05, 2000, 0.05, 2048), (1.6, 0.3, 50, 0.02, 20)]:
        p = base()
        p.ny, p.r, p.gamma, p.u_lid = ny, r, g, U
        capi.prc_params_from_re(p, re_)
        po = O.with_re(O.params(64, ny, r, g, 1.0, u_lid=U), re_)
        assert abs(p.omega_nu - po.omega_nu) < 1e-15 * po.omega_nu


def test_cavity_64x32_relaxation_rate():
    # Re = 100 with H = 64 dx and U = 0.05: nu = 0.032, omega = 1/(3 nu + 1/2)
    p = base()
    p.r, p.u_lid = 2.0, 0.05
    capi.prc_params_from_re(p, 100.0)
    assert abs(p.omega_nu - 1.0 / (0.096 + 0.5)) < 1e-14


@pytest.mark.parametrize("field,value", [
    ("nx", 2), ("ny", 0), ("r", 0.0), ("r", -1.0), ("gamma", 0.0), ("gamma", 1.5),
    ("omega_nu", 2.0), ("omega_xi", 0.0), ("u_lid", 0.6), ("rho0", 0.0), ("bc", 3),
    ("storage", 4), ("corrections", 8), ("frame", 5),
])
def test_validation_rejects(field, value):
    p = base()
    setattr(p, field, value)
    with pytest.raises(capi.PrcError) as e:
        capi.prc_validate(p)
    assert e.value.status == capi.PRC_EINVAL
    assert capi.prc_last_error()
    assert capi.lib().prc_state_bytes(p) == 0


def test_lid_speed_limit_uses_rectangular_sound_speed():
    p = base()
    p.r, p.u_lid = 0.5, 0.3   # below 1/sqrt(3) but above 0.5/sqrt(3)
    with pytest.raises(capi.PrcError):
        capi.prc_validate(p)
    p.u_lid = 0.28
    capi.prc_validate(p)


@pytest.mark.parametrize("storage,elem", [(0, 8), (1, 4), (2, 2), (3, 2)])
def test_layout_and_sizes(storage, elem):
    p = base()
    p.nx, p.ny, p.storage = 1000, 37, storage
    row, plane = capi.prc_layout(p)
    # every element (a, j, i) lies inside the buffer and no two coincide
    offs = sorted(a * plane + j * row + i for a in range(9) for j in range(37) for i in (0, 999))
    assert offs[0] == 0 and len(set(offs)) == len(offs)
    assert (offs[-1] + 1) * elem <= capi.prc_state_bytes(p)
    assert (row * elem) % 256 == 0 and (plane * elem) % 256 == 0
    assert capi.prc_scratch_bytes(p) > 0


def test_from_re_rejects_bad_input():
    p = base()
    p.u_lid = 0.0
    with pytest.raises(capi.PrcError):
        capi.prc_params_from_re(p, 100.0)
    p.u_lid = 0.05
    with pytest.raises(capi.PrcError):
        capi.prc_params_from_re(p, -1.0)


def test_set_tile_validates_without_gpu():
    p = base()
    capi.prc_set_tile(p, 1)
    capi.prc_set_tile(p, 7)      # two steps per launch
    capi.prc_set_tile(p, -1)
    with pytest.raises(capi.PrcError):
        capi.prc_set_tile(p, 9)
    with pytest.raises(capi.PrcError):
        capi.prc_set_tile(p, -2)
    p.storage = capi.PRC_F64
    capi.prc_set_tile(p, 5)      # every shape runs every storage
    capi.prc_set_tile(p, -1)


# ---- batches: host-side argument checks (nothing is launched) -------------

def test_batch_host_checks():
    b = capi.prc_batch_create(capi.PRC_F32, capi.PRC_BC_CAVITY)
    try:
        assert capi.prc_batch_count(b) == (0, 0)
        p = base()
        fake_a, fake_b, fake_u = 256 * 1000, 256 * 3000, 256 * 5000  # never dereferenced
        with pytest.raises(capi.PrcError):           # storage differs from the batch's
            q = p.copy()
            q.storage = capi.PRC_F64
            capi.prc_batch_add(b, q, fake_a, fake_b, fake_u)
        with pytest.raises(capi.PrcError):           # boundary type differs
            q = p.copy()
            q.bc = capi.PRC_BC_PERIODIC
            capi.prc_batch_add(b, q, fake_a, fake_b, fake_u)
        with pytest.raises(capi.PrcError):           # misaligned buffer
            capi.prc_batch_add(b, p, fake_a + 4, fake_b, fake_u)
        with pytest.raises(capi.PrcError):           # same buffer twice
            capi.prc_batch_add(b, p, fake_a, fake_a, fake_u)
        with pytest.raises(capi.PrcError):           # invalid problem
            q = p.copy()
            q.gamma = 0.0
            capi.prc_batch_add(b, q, fake_a, fake_b, fake_u)
        assert capi.prc_batch_count(b) == (0, 0)
        assert capi.prc_batch_add(b, p, fake_a, fake_b, fake_u) == 0
        assert capi.prc_batch_add(b, p, fake_b, fake_a, fake_u) == 1
        assert capi.prc_batch_count(b) == (2, 2)
        capi.prc_batch_remove(b, 0)
        assert capi.prc_batch_count(b) == (2, 1)
        for bad in (0, 2, -1):                        # removed, unknown, negative
            with pytest.raises(capi.PrcError):
                capi.prc_batch_remove(b, bad)
        with pytest.raises(capi.PrcError):
            capi.prc_batch_step(b, 3)                 # odd step counts are refused
        with pytest.raises(capi.PrcError):
            capi.prc_batch_solve(b, 1e-6, 100, 250)   # max_steps not a multiple
        with pytest.raises(capi.PrcError):
            capi.prc_batch_solve(b, 1e-6, 101, 202)   # odd check interval
        for t in (-1, 8):
            with pytest.raises(capi.PrcError):
                capi.prc_batch_set_tile(b, t)
        capi.prc_batch_set_tile(b, 2)
        capi.prc_batch_set_tile(b, 6)      # two steps per launch
        capi.prc_batch_set_tile(b, 7)      # 64 x 16, two steps per launch
    finally:
        capi.prc_batch_destroy(b)


@pytest.mark.parametrize("storage,bc", [(4, 0), (-1, 0), (1, 3)])
def test_batch_create_rejects(storage, bc):
    with pytest.raises(capi.PrcError):
        capi.prc_batch_create(storage, bc)


def serve_cfg(**kw):
    c = capi.prc_serve_config(storage=capi.PRC_F32, bc=capi.PRC_BC_CAVITY, tol=1e-6,
                              check_every=100, max_steps=1000, hbm_budget=1 << 24,
                              max_active=0, tile=-1)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw", [dict(check_every=99), dict(check_every=0), dict(max_steps=150),
                                dict(tol=-1.0), dict(tile=8), dict(hbm_budget=100),
                                dict(storage=7), dict(bc=4)])
def test_serve_rejects_bad_config(kw):
    with pytest.raises(capi.PrcError) as e:
        capi.prc_serve(serve_cfg(**kw), [])
    assert e.value.status == capi.PRC_EINVAL


def test_serve_rejects_unordered_arrivals():
    p = base()
    reqs = [capi.prc_request(1.0, p, None, None), capi.prc_request(0.5, p, None, None)]
    with pytest.raises(capi.PrcError) as e:
        capi.prc_serve(serve_cfg(), reqs)
    assert "non-decreasing" in str(e.value)


def test_serve_empty_trace_is_a_no_op():
    assert capi.prc_serve(serve_cfg(), []) == []


def test_state_size_limit_is_4_gib():
    """Byte offsets into a state are 32-bit: the largest accepted state is the
    last that fits 4 GiB, one more row is rejected."""
    p = base()
    p.nx, p.storage = 16384, capi.PRC_F32
    row, _ = capi.prc_layout(p)
    ny_max = (2 ** 32 - 1) // (row * 4)
    p.ny = ny_max
    assert capi.prc_state_bytes(p) <= 2 ** 32 - 1
    p.ny = ny_max + 1
    with pytest.raises(capi.PrcError):
        capi.prc_validate(p)


@pytest.mark.parametrize("kw", [dict(check_every=0), dict(max_steps=-1),
                                dict(tol=-1.0), dict(tol=float("nan"))])
def test_solve_rejects_bad_arguments_before_launching(kw):
    p = base()
    args = dict(tol=1e-6, check_every=100, max_steps=1000)
    args.update(kw)
    with pytest.raises(capi.PrcError) as e:
        capi.prc_solve(p, 256 * 1000, 256 * 2000, 256 * 3000, 256 * 4000, args["tol"],
                       args["check_every"], args["max_steps"])
    assert e.value.status == capi.PRC_EINVAL


@pytest.mark.parametrize("a,b,n", [(0, 256 * 2000, 1), (256 * 1000, 256 * 1000, 1),
                                   (256 * 1000 + 4, 256 * 2000, 1), (256 * 1000, 256 * 2000, -1)])
def test_step_rejects_bad_buffers_before_launching(a, b, n):
    with pytest.raises(capi.PrcError) as e:
        capi.prc_step(base(), a, b, n)
    assert e.value.status == capi.PRC_EINVAL


def test_tile_info():
    shapes = [capi.prc_tile_info(t) for t in range(10)]
    assert shapes[0] == (64, 4, 1) and shapes[8] == (32, 32, 2)
    assert [s[2] for s in shapes] == [1] * 5 + [2] * 4 + [0]  # 0: resident, any count
    assert shapes[9][:2] == (64, 32)
    with pytest.raises(capi.PrcError):
        capi.prc_tile_info(10)


def test_resident_tile_needs_a_device():
    """Whether the resident sweep fits is a property of the device (its
    compute units and LDS): without one it is refused."""
    with pytest.raises(capi.PrcError):
        capi.prc_set_tile(base(), 9)


def test_batch_tile_range():
    b = capi.prc_batch_create(capi.PRC_F64, capi.PRC_BC_CAVITY)
    try:
        capi.prc_batch_set_tile(b, 5)    # two steps per launch, FP64 included
        capi.prc_batch_set_tile(b, 4)
        capi.prc_batch_set_tile(b, 7)    # 64 x 16, two steps per launch
        with pytest.raises(capi.PrcError):
            capi.prc_batch_set_tile(b, 8)  # not a batch shape
    finally:
        capi.prc_batch_destroy(b)
