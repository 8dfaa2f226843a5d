"""Helpers shared by the GPU tests: build a library System and the matching
oracle model from one configuration and one set of seeded inputs."""
import sys

import numpy as np

import workloads as W


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def make_pair(cfg, precision="f64", n_orb=None, taylor_order=4, **over):
    """(System, oracle Model, oracle State, inputs) for one configuration."""
    import torch
    from paper_0812_2801_amd import binding as B
    from oracle import Model, dynamics
    if n_orb is not None:
        cfg = cfg.replace(n_orb=n_orb)
    cfg = cfg.replace(**over) if over else cfg
    inp = W.make_inputs(cfg)
    p, keep = B.params_from_config(cfg, inp["pos"], precision=precision,
                                   taylor_order=taylor_order)
    sysm = B.System(p, keep)
    sysm.set_state(torch.from_numpy(inp["psi"].reshape(cfg.n_orb, -1)))
    m = Model.from_config(cfg, taylor_order=taylor_order)
    st = dynamics.init_state(m, inp["psi"], inp["pos"])
    return sysm, m, st, inp, cfg


def to_np(t):
    return t.detach().cpu().numpy()
