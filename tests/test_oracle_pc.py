"""Pins of the oracle's capillary-pressure sweep (oracle/pc_sweep.py).

Drainage of a slit between two solid plates of aperture h (fluid rows): the
capillary entry pressure of a slit is 2 sigma cos(theta) / h, at most
2 sigma / h for any contact angle of a wetted wall, with sigma the model's
surface tension (sigma_0 of tests/golden/kappa.json, measured on the
oracle by Laplace's law at G = 3, tau = 1, kappa = 0).  At a reservoir
pressure difference of 1.5 times that bound the oil must fill the slit and
then stop at the membrane, whose entry pressure (0.3) is well above the
level: a steady state with the sample almost free of water and no oil past
the membrane.  The box and the level follow from the protocol's own
definitions, checked here too."""
import json
import os

import numpy as np

import workloads as W
from oracle.pc_sweep import pc_sweep, sweep_box, bulk_pressure

GOLD = os.path.join(os.path.dirname(__file__), "golden", "kappa.json")


def test_sweep_box_layout():
    cls = np.zeros((3, 4, 5), np.uint8)
    cls[1, 2, 3] = 1
    box, sample = sweep_box(cls, buffer_in=4, membrane=2, buffer_out=3, side_walls=True)
    assert box.shape == (5, 6, 4 + 5 + 2 + 3)
    assert np.all(box[0] == 1) and np.all(box[:, -1] == 1)           # the frame
    assert np.all(box[1:-1, 1:-1, :4] == 0)                          # inlet buffer
    assert np.array_equal(box[1:-1, 1:-1, 4:9], cls)                 # the domain
    assert np.all(box[1:-1, 1:-1, 9:11] == 2)                        # membrane
    assert np.all(box[1:-1, 1:-1, 11:] == 0)                         # outlet buffer
    assert sample.sum() == cls.size - 1 and not sample[2, 3, 7]


def test_slit_fills_above_the_entry_bound_and_stops_at_the_membrane():
    sigma = json.load(open(GOLD))["sigma0"]
    su = W.pc_sweep_setup()
    p = su["model"]
    m, G = p.m_minor, p.G
    h, L = 10, 8
    cls = np.zeros((1, h + 2, L), np.uint8)
    cls[:, 0, :] = cls[:, -1, :] = 1
    target = 1.5 * 2.0 * sigma / h
    p_out = bulk_pressure(1.0, m, G)
    # inlet oil density whose bulk pressure exceeds the outlet's by `target`
    rho = (3.0 * (p_out + target) - m) / (1.0 + G * m)
    keep = []
    out = pc_sweep(cls, p, su["membrane_table"], [rho], buffer_in=4, membrane=2, buffer_out=2,
                   side_walls=False, membrane_phi=su["membrane_phi"], check_every=100,
                   max_steps=1500, tol=1e-3, keep=keep)
    assert abs(out["pc"][0] - target) < 1e-12
    assert out["converged"][0]
    assert out["sw"][0] < 0.15, out
    f = keep[-1]
    # no oil beyond the membrane (outlet buffer: the last two planes)
    assert f["rho_o"][:, 1:-1, -2:].max() < 0.05
    # the slit holds oil up to the interface's width (about two voxels) before the membrane
    assert f["rho_o"][:, 1:-1, 4:4 + L - 2].min() > 0.5
