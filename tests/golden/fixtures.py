"""Loaders for the hand-derived fixtures in this folder."""
import json
import os

import numpy as np

import scenegen

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    with open(os.path.join(HERE, name)) as f:
        d = json.load(f)
    f32 = lambda k: np.asarray(d[k], np.float32)  # noqa: E731
    scene = scenegen.Scene(width=d["width"], height=d["height"], spp=d["spp"],
                           path_offsets=np.asarray(d["path_offsets"], np.int64), pos=f32("pos"),
                           dir_in=f32("dir_in"), dir_out=f32("dir_out"), albedo=f32("albedo"),
                           l_sun=f32("l_sun"), dir_env=f32("dir_env"), l_env=f32("l_env"),
                           l_phase=f32("l_phase"), e_cam=f32("e_cam"))
    return scene, d
