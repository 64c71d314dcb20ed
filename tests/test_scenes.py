"""Seeded scene inputs: the frames do not depend on how they were rendered.

A process that holds the GPU open renders its scenes in-process rather than
in forked workers; both ways must give the same bytes, so that a GPU test
sees the inputs the benchmark and the oracle pins see."""
import numpy as np

import scenes


def test_gpu_not_open_here():
    assert scenes._gpu_open() is False


def test_serial_and_pooled_rendering_agree():
    a = scenes.room_scene(n_obj=3, n_views=6, W=96, H=72, seed=2, room=4.0)
    b = scenes.room_scene(n_obj=3, n_views=6, W=96, H=72, seed=2, room=4.0)
    scenes._render_frames(b, depth_frac=0.005, seed=2, workers=1)
    assert len(a.frames) == len(b.frames) == 6
    for (ca, ra, ma, da), (cb, rb, mb, db) in zip(a.frames, b.frames):
        assert np.array_equal(ra, rb) and np.array_equal(ma, mb)
        assert np.array_equal(da, db)
        assert np.array_equal(np.asarray(ca["T_wc"]), np.asarray(cb["T_wc"]))
