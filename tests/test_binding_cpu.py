"""The Python binding hands raw tensor pointers to the library, so it must
refuse, before any call into it, every tensor of the wrong dtype, shape or
device or not contiguous: a host tensor passed to a kernel as a device
pointer would fault the GPU.  Checked on the CPU: the objects are built
without their constructors on the "meta" device (tensors with a shape and
no storage), and the library is replaced by a stub that fails the test if
any call reaches it."""
import contextlib
import ctypes

import pytest
import torch

import paper_1708_02645_amd as q

META = torch.device("meta")
B, N = 5, 8


class _Stub:
    def __getattr__(self, name):
        if name.endswith("_workspace_bytes"):
            return lambda *a: 4096

        def reached(*a):
            raise AssertionError("library reached: " + name)
        return reached


@pytest.fixture(autouse=True)
def stub(monkeypatch):
    """Library calls fail the test; device and stream selection are no-ops,
    so a missing check would run on into the stub instead of stopping at
    torch's own refusal of the meta device."""
    monkeypatch.setattr(q, "lib", lambda: _Stub())
    monkeypatch.setattr(q, "_mlp_lib", lambda: _Stub())
    monkeypatch.setattr(q, "_stream_ptr", lambda torch_, device, stream: (ctypes.c_void_p(0), None))
    monkeypatch.setattr(torch.cuda, "device", lambda d: contextlib.nullcontext())


def _m(*shape, dtype=torch.float32):
    return torch.empty(shape, dtype=dtype, device=META)


def _spline():
    s = object.__new__(q.Spline)
    s._torch, s.device, s.norb, s.dtype, s._h = torch, META, N, "f32", None
    return s


def _bad_variants(t):
    """The tensor on the host, with another dtype, with another shape, and
    not contiguous."""
    yield torch.empty(t.shape, dtype=t.dtype)
    yield torch.empty(t.shape, dtype=torch.float64 if t.dtype != torch.float64 else torch.float32, device=META)
    yield torch.empty((t.shape[0] + 1,) + tuple(t.shape[1:]), dtype=t.dtype, device=META)
    if t.dim() >= 2:
        yield torch.empty(tuple(t.shape[::-1]), dtype=t.dtype, device=META).transpose(0, -1)


def _each_bad(good):
    """Every tuple that replaces one member of `good` with a bad variant."""
    for i, t in enumerate(good):
        for b in _bad_variants(t):
            yield tuple(b if j == i else u for j, u in enumerate(good))


def test_spline_outputs_checked():
    s = _spline()
    pos = _m(B, 3, dtype=torch.float64)
    vgl = (_m(B, N), _m(B, 3, N), _m(B, N))
    vgh = (_m(B, N), _m(B, 3, N), _m(B, 6, N))
    calls = [lambda o: s.eval_vgl(pos, out=o), lambda o: s.eval_vgl_sorted(pos, out=o),
             lambda o: s.autotune(pos, out=o), lambda o: s.autotune_sorted(pos, out=o)]
    for call in calls:
        for bad in _each_bad(vgl):
            with pytest.raises(ValueError):
                call(bad)
    for call in (lambda o: s.eval_vgh(pos, out=o), lambda o: s.eval_vgh_sorted(pos, out=o),
                 lambda o: s.autotune_vgh(pos, out=o)):
        for bad in _each_bad(vgh):
            with pytest.raises(ValueError):
                call(bad)
    for call in (lambda o: s.eval_v(pos, out=o), lambda o: s.eval_v_sorted(pos, out=o)):
        for (bad,) in _each_bad((_m(B, N),)):
            with pytest.raises(ValueError):
                call(bad)
    ainv = _m(B, N)
    for call in (s.eval_ratio_vgl, s.eval_ratio_vgl_sorted):
        for (bad,) in _each_bad((_m(B, 5),)):
            with pytest.raises(ValueError):
                call(pos, ainv, out=bad)
    for (bad,) in _each_bad((pos,)):
        with pytest.raises(ValueError):
            s.eval_vgl(bad, out=vgl)
    for (bad,) in _each_bad((ainv,)):
        if bad.shape[0] == B + 1 and bad.device == META:
            continue  # a taller inverse is allowed
        with pytest.raises(ValueError):
            s.eval_ratio_v(pos, bad, out=_m(B))
    with pytest.raises(ValueError):
        s.eval_vgl_sorted(pos, out=vgl, workspace=torch.empty(4096, dtype=torch.uint8))  # host workspace
    with pytest.raises(ValueError):
        s.eval_vgl_sorted(pos, out=vgl, workspace=_m(4095, dtype=torch.uint8))  # short workspace


def test_plan_outputs_checked():
    s = _spline()
    pos = _m(B, 3, dtype=torch.float64)
    good = (_m(B, N), _m(B, 3, N), _m(B, N))
    for bad in _each_bad(good):
        with pytest.raises(ValueError):
            q.Plan([s], [pos], outs=[bad])
    with pytest.raises(ValueError):
        q.Plan([s], [pos], outs=[good, good])


def test_delayed_update_checked():
    d = object.__new__(q.DelayedUpdate)
    d._torch, d.device, d.n, d.delay, d.walkers, d._h = torch, META, N, 4, B, None
    ainv = _m(B, N, N)
    k = _m(B, dtype=torch.int32)
    V = _m(B, N)
    G, L = _m(B, 3, N), _m(B, N)
    for bad in _each_bad((k, V)):
        with pytest.raises(ValueError):
            d.ratio(ainv, *bad)
        with pytest.raises(ValueError):
            d.accept(ainv, *bad)
    for bad in _each_bad((G, L)):
        with pytest.raises(ValueError):
            d.ratio(ainv, k, V, *bad)
    for (bad,) in _each_bad((_m(B, 5),)):
        with pytest.raises(ValueError):
            d.ratio(ainv, k, V, G, L, out=bad)
        with pytest.raises(ValueError):
            d.accept_ratio(ainv, k, V, k, V, G, L, out=bad)
    for (bad,) in _each_bad((k,)):
        with pytest.raises(ValueError):
            d.ratio(ainv, k, V, walkers=bad)
    with pytest.raises(ValueError):
        d.flush(torch.empty((B, N, N)))


def test_jastrow_checked():
    j = object.__new__(q.Jastrow)
    j._torch, j.device, j.n_elec, j.n_ion, j._h = torch, META, 6, 0, None
    R = _m(B, 3, 8)
    k = _m(B, dtype=torch.int32)
    r = _m(B, 3, dtype=torch.float64)
    for (bad,) in _each_bad((_m(B, 5),)):
        with pytest.raises(ValueError):
            j.move(R, k, r, out=bad)
    for bad in _each_bad((_m(B), _m(B, 3, 6), _m(B, 6))):
        with pytest.raises(ValueError):
            j.evaluate(R, out=bad)
    with pytest.raises(ValueError):
        j.move(torch.empty((B, 3, 8)), k, r)


def test_surrogate_checked():
    m = object.__new__(q.SurrogateMLP)
    m._torch, m.device, m.norb, m._h, m._ws = torch, META, N, None, {}
    pos = _m(B, 3, dtype=torch.float64)
    vgl = (_m(B, N), _m(B, 3, N), _m(B, N))
    for bad in _each_bad(vgl):
        with pytest.raises(ValueError):
            m.forward(pos, out=bad)
        with pytest.raises(ValueError):
            m.eval_vgl(pos, out=bad)
        with pytest.raises(ValueError):
            m.grad(pos, bad)
        with pytest.raises(ValueError):
            m.train_step(pos, bad, 1e-3)
    for (bad,) in _each_bad((pos,)):
        with pytest.raises(ValueError):
            m.forward(bad, out=vgl)


def test_module_functions_checked():
    with pytest.raises(ValueError):
        q.det_update(torch.empty((B, N, N)), torch.empty(B, dtype=torch.int32), torch.empty((B, N)))
    with pytest.raises(ValueError):
        q.probe_stream_read(torch.empty(1024, dtype=torch.uint8))
