"""Host-side bounds check of the tables the kernels read through
(opf_check_network, which opf_load_network also runs before it changes
anything): node CSR over line terminals and devices, the node clusters of
the tiled sweep with their line tables, ramp, DC link and change indices.
Runs on the CPU: the check touches no device."""
import numpy as np
import pytest

from paper_2410_17203_amd import synth
from paper_2410_17203_amd.binding import OpfError, check_network
from tests.test_gpu_parity import make

# cluster limits of the tiled sweep (lines and devices one cluster holds)
TILE_LINES = 128
TILE_DEV = 128


@pytest.mark.parametrize("name", ["tiny", "medium", "wide_T", "three_slots", "edge", "curtailable",
                                  "hvdc", "changes", "changes_dc"])
def test_tables_of_the_parity_instances_pass(name):
    assert check_network(make(name)) is True


def test_batch_instances_and_the_large_grid_pass():
    for x in synth.batched()[:16]:
        assert check_network(x, dtype="f32") is True
    assert check_network(synth.config("large"), dtype="f32") is True


def star(n_lines, n_loads_at_hub=1):
    """Node 0 joined to nodes 1..n_lines, and the last of them to one more
    node; a generator at node 0, n_loads_at_hub loads at node 0 and one at
    every other node."""
    N = n_lines + 2
    f = lambda v: np.asarray(v, np.float64)
    line_from = np.r_[np.zeros(n_lines, np.int32), [n_lines]].astype(np.int32)
    line_to = np.r_[np.arange(1, n_lines + 1), [n_lines + 1]].astype(np.int32)
    L = len(line_from)
    load_node = np.r_[np.zeros(n_loads_at_hub, np.int32), np.arange(1, N)].astype(np.int32)
    D = len(load_node)
    return synth.Instance(
        name="star", N=N, T=2, K=1, line_from=line_from, line_to=line_to,
        line_sus=f([10.0] * L), line_cap=f([1.0] * L), outage=np.asarray([L - 1], np.int32),
        gen_node=np.zeros(1, np.int32), gen_c2=f([0.05]), gen_c1=f([20.0]),
        gen_pmin=np.zeros((1, 2)), gen_pmax=np.full((1, 2), 1e3), gen_ramp=f([np.inf]),
        load_node=load_node, load_d=np.full((D, 2), 0.01),
        bat_node=np.zeros(0, np.int32), bat_P=f([]), bat_dur=f([]), bat_eta=f([]),
        bat_alpha=f([]), meta={})


def test_cluster_limits_at_the_boundary():
    # a node with exactly as many lines (devices) as a cluster holds still
    # gets a cluster; one more and the tiled sweep is not available
    assert check_network(star(TILE_LINES)) is True
    assert check_network(star(TILE_LINES + 1)) is False
    assert check_network(star(4, n_loads_at_hub=TILE_DEV - 1)) is True  # + the generator
    assert check_network(star(4, n_loads_at_hub=TILE_DEV)) is False
    assert check_network(make("hub")) is False


def test_invalid_networks_are_rejected_with_a_reason():
    x = synth.config("tiny")
    x.line_to = np.array(x.line_to)
    x.line_to[3] = x.N
    with pytest.raises(OpfError, match="line node index out of range"):
        check_network(x)
    y = synth.config("tiny")
    y.K = 1
    y.outage = np.asarray([len(y.line_from)], np.int32)
    with pytest.raises(OpfError):
        check_network(y)
    z = make("changes")
    z.chg_k = np.r_[z.chg_k, z.chg_k[:1]]
    z.chg_line = np.r_[z.chg_line, z.chg_line[:1]]
    z.chg_sus = np.r_[z.chg_sus, z.chg_sus[:1]]
    z.chg_cap = np.r_[z.chg_cap, z.chg_cap[:1]]
    with pytest.raises(OpfError, match="changed twice"):
        check_network(z)
