"""Writes the stored model files tests/golden/model_<tag>.json.

Each file completes a seeded random network (paper_2107_11311_amd.inputs) with
  * a per-species input normalisation x0 = (G - shift) * scale, shift = mean and
    scale = 1/std of the oracle's descriptors of that species on frame 0 of the
    workload (std < 1e-12 -> scale 1), and
  * one output-layer scale factor chosen so that the oracle's force RMS on frame
    0 is 1 eV/A (forces are linear in the last weight matrix).
The paper trains its networks on DFT data that is not available here; these
files make random networks produce inputs and forces of a sensible magnitude.
Only the oracle computes anything here.

Usage: python tests/golden/make_models.py [tag ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2107_11311_amd import inputs as I  # noqa: E402

# tag -> (workload whose network is used, workload whose frame 0 is fitted, net seed offset)
TAGS = {
    "water64": ("water64", "water64", 0),
    "water4096": ("water4096", "water4096", 0),
    "water4096_ref": ("water4096", "water4096", 1000),
    "lisio120k": ("lisio120k", "lisio120k", 0),
    "student": ("student", "water4096", 0),
    # the distillation teacher: the water4096 network reduced to a
    # 20-16-16-1 network on the student's descriptor components (see
    # paper_2107_11311_amd.inputs.sub_network), force RMS 1 eV/A on frame 0
    "student_teacher": ("water4096", "water4096", 0),
}
SUB_NETWORK = {"student_teacher": {"radial_order": 6, "angular_order": 2, "hidden": [16, 16]}}


def fit(tag: str) -> dict:
    cfg, frame_cfg, seed_off = TAGS[tag]
    t0 = time.time()
    model = I.raw_model(cfg, seed_off)
    sub = SUB_NETWORK.get(tag)
    if sub:
        model = I.sub_network(model, sub["radial_order"], sub["angular_order"], sub["hidden"])
    sysm = I.make_system(frame_cfg)
    G = oracle.descriptors(model, sysm.pos, sysm.species, sysm.box, sysm.pbc)
    shift, scale = [], []
    for t in range(model.n_species):
        Gt = G[sysm.species == t]
        mu = Gt.mean(0)
        sd = Gt.std(0)
        sd = np.where(sd < 1e-12, 1.0, sd)
        shift.append(mu.tolist())
        scale.append((1.0 / sd).tolist())
    norm = dict(config=cfg, frame=frame_cfg, net_seed_offset=seed_off, shift=shift, scale=scale,
                out_scale=1.0)
    if sub:
        norm["sub_network"] = sub
    m1 = I.apply_normalisation(model, norm)
    _, _, F = oracle.energy_forces(m1, sysm.pos, sysm.species, sysm.box, sysm.pbc)
    rms = float(np.sqrt(np.mean(F * F)))
    norm["out_scale"] = 1.0 / rms
    norm["force_rms_unscaled"] = rms
    norm["n_atoms"] = int(sysm.pos.shape[0])
    norm["fit_seconds"] = round(time.time() - t0, 1)
    return norm


def main(tags):
    for tag in tags:
        norm = fit(tag)
        with open(I.model_file(tag), "w") as f:
            json.dump(norm, f, indent=1)
        print(tag, "force rms before scaling", norm["force_rms_unscaled"], "seconds", norm["fit_seconds"],
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or [t for t in TAGS if t != "lisio120k"])
