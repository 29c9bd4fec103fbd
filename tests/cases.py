"""Shared workload cases of the GPU tests (seeded, synthetic)."""
import math

import numpy as np

import fte_workloads as W

AU = W.AU
DEG = W.DEG


def near_observers(params):
    """The tiny Parker workload's own observer (1 au, 60 ten-minute bins)
    closes before 100 keV protons can arrive along the spiral, so the parity
    tests add observers on the connected field line at 0.3 and 0.6 au and
    extend the time bins over the whole 5,000-step run."""
    om, V = W.OMEGA_SYNODIC, 400e3
    obs = [(r * AU, 90 * DEG, W.OMEGA_SYNODIC * (1.0 - r) * AU / V, 0.05 * AU, 10 * DEG, 10 * DEG)
           for r in (0.3, 0.6, 1.0)]
    del om
    return dict(params, observers=obs, n_t=84)


def amr_cir_case(n_levels=3, kperp=0.05, model="eq5", n_snap=3):
    n1, bx = (32, 8, 32), (8, 4, 8)
    rng = np.random.default_rng(1)
    marks = {}

    def refine(L, I, J, K):
        key = (L, I, J, K)
        if key not in marks:
            marks[key] = rng.random() < 0.4
        return marks[key]

    leaves = W.amr_leaves(n1, bx, n_levels, refine)
    g = W.grid_desc(1, 0.1 * AU, math.log(12.0) / n1[0], 60 * DEG, 60 * DEG / n1[1], 0.0, 2 * math.pi / n1[2], n1,
                    bx, leaves, n_levels, n_snap=n_snap, t_s0=0.0, dt_s=3600.0)
    p = dict(mass=W.M_P, dmm_model=model, lambda_ref=0.05 * AU, q=5 / 3, eps=0.048, mu_floor=1e-4,
             kperp_ratio=kperp, dt=20.0, r_in=0.09 * AU, r_out=1.15 * AU, seed=12345, run_id=3,
             observers=[(0.3 * AU, 90 * DEG, p * DEG, 0.1 * AU, 20 * DEG, 40 * DEG) for p in (0, 90, 200)],
             t_ref=0.0, dT=400.0, n_t=9, n_batch=16, precision="fp64",
             e_min=20 * W.KEV, dlne=math.log(10) / 8, n_e=8)
    inj = dict(r=0.15 * AU, th_lo=70 * DEG, th_hi=110 * DEG, ph_lo=0.0, ph_hi=2 * math.pi, e_lo=30 * W.KEV,
               e_hi=300 * W.KEV, gamma_inj=3.0, w0=2.0, pid0=1000, n_total=777, k0=5, n_inj_steps=120)
    return p, g, inj
