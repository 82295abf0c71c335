"""The seeded generators: determinism, shapes and value laws."""
import numpy as np

import instancegen


def test_deterministic_and_shapes():
    a = instancegen.draw_config("fourier_n65536", 0)
    b = instancegen.draw_config("fourier_n65536", 0)
    assert np.array_equal(a.omega, b.omega) and np.array_equal(a.values, b.values)
    assert a.omega.shape == (16384,) and np.all(np.diff(a.omega) > 0)
    assert a.support.shape == (256,) and len(set(a.support)) == 256
    assert np.iscomplexobj(a.values) and a.noise.shape == (16384,)
    c = instancegen.draw_config("fourier_n65536", 1)
    assert not np.array_equal(a.omega, c.omega)


def test_value_laws():
    h = instancegen.draw_instance("H", 4096, 1024, 500, "pm_u12", None, 3)
    assert np.all((np.abs(h.values) >= 1) & (np.abs(h.values) <= 2))
    assert h.noise is None
    i = instancegen.draw_instance("H", 64, 32, 8, "int", None, 3)
    assert np.all(i.values == np.round(i.values)) and np.all(i.values != 0)


def test_batch_descriptors():
    b = instancegen.draw_batch(64)
    for i, inst in enumerate(b):
        assert inst.cls == ("F" if i % 2 == 0 else "H")
        assert 1 << 10 <= inst.N <= 1 << 14 and inst.M == inst.N // 4
        assert 8 <= inst.K <= inst.M // 8


def test_stream_descriptors():
    t, insts = instancegen.draw_stream(50)
    assert np.all(np.diff(t) > 0)
    for inst in insts:
        assert inst.N // 8 <= inst.M <= inst.N // 4 and 16 <= inst.K <= inst.M // 16
