"""Instances for the derivative tests: small networks with tight line
capacities, generator limits and cheap generators, so that line, generator
and ramp clips become active within tens of iterations (otherwise the
capacity and limit derivatives of a short unrolled run are all zero)."""
import numpy as np

from paper_2410_17203_amd import synth


def tight(name="adj", N=14, L=20, G=4, D=10, B=2, T=6, K=3, seed=77):
    inst = synth.make_instance(name, N=N, L=L, G=G, D=D, B=B, T=T, K=K, seed=seed)
    inst.line_cap = np.asarray(inst.line_cap) * 0.3
    inst.gen_pmax = np.asarray(inst.gen_pmax) * 0.8
    inst.gen_c1 = np.asarray(inst.gen_c1) * 0.02
    return inst


def weights(inst, seed=0):
    """Fixed N(0, 1) weights on the device powers [G+D+B, T]."""
    J = len(inst.gen_node) + len(inst.load_node) + len(inst.bat_node)
    return np.random.default_rng(seed).normal(size=(J, int(inst.T)))
