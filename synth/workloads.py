"""Named workloads: volume, detector and pose recipes of the benchmarks.

small    : 64^3 CT at 1 mm, 64 x 64 detector at 2.0 mm, SDD 1000 mm, one pose
           with angles in +-pi/8 and shifts in +-10 mm (4096 rays).
ct512    : 512 x 512 x 133 CT at 0.7 x 0.7 x 2.5 mm, 256 x 256 detector at
           1.4 mm, SDD 1020 mm, poses with angles in +-pi/6 and shifts in
           +-30 mm; 1 pose or 256 poses per launch.
ct512_grad : same CT, 200 x 200 detector at 1.4 mm, 64 poses, negative-NCC
           loss against a target rendered at a seeded ground-truth pose.
"""

from __future__ import annotations

from dataclasses import dataclass
import math


@dataclass(frozen=True)
class Workload:
    name: str
    phantom: str
    height: int
    width: int
    pitch: float          # detector pixel pitch, mm (rows and columns)
    sdd: float
    max_angle: float
    max_shift: float
    n_poses: int


WORKLOADS = {
    "small": Workload("small", "small", 64, 64, 2.0, 1000.0, math.pi / 8, 10.0, 1),
    "ct512_1": Workload("ct512_1", "ct512", 256, 256, 1.4, 1020.0, math.pi / 6, 30.0, 1),
    "ct512_256": Workload("ct512_256", "ct512", 256, 256, 1.4, 1020.0, math.pi / 6, 30.0, 256),
    "ct512_grad": Workload("ct512_grad", "ct512", 200, 200, 1.4, 1020.0, math.pi / 6, 30.0, 64),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
