"""Ragged work lists on the GPU: pairs of mixed sizes (and masked/unmasked)
searched as one captured launch must give, pair for pair, exactly what the
batched search gives on the same scans, on every replay, and must read the
scans anew at each launch."""
import numpy as np
import pytest
import torch

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import fmbym, synth, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SIZES = ("pair128", "batch256", "batch512")


def _searches():
    return {name: fmbym.Search(max_batch=8, **workloads.search_kwargs(name)) for name in SIZES}


def _work_list(names, masked_every=0, split="val"):
    """Device tensors for each pair of the list; masks on every k-th pair."""
    pairs, count = [], {}
    rng = np.random.Generator(np.random.PCG64(5))
    for i, name in enumerate(names):
        k = count.get(name, 0)
        count[name] = k + 1
        f, g, _ = synth.make_batch(name, 1, split=split, start=k)
        q = [torch.from_numpy(f[0]).to(DEV), torch.from_numpy(g[0]).to(DEV)]
        if masked_every and i % masked_every == masked_every - 1:
            n = f.shape[-1]
            q += [torch.from_numpy(rng.uniform(0.2, 1.0, (n, n)).astype(np.float32)).to(DEV)
                  for _ in range(2)]
        pairs.append(q)
    return pairs


def _eager_poses(searches, names, pairs):
    """The batched search of each pair alone (batch 1), in list order."""
    out = torch.empty(len(pairs), 3, device=DEV)
    for i, (name, q) in enumerate(zip(names, pairs)):
        s = searches[name]
        args = [t[None] for t in q] + [None] * (4 - len(q))
        out[i] = s.forward(*args, surfaces=False)["pose"][0]
    return out


NAMES = ["batch256", "pair128", "batch512", "pair128", "batch256", "pair128", "batch512", "pair128",
         "batch256"]


def test_ragged_equals_batched_search_on_every_replay():
    searches = _searches()
    pairs = _work_list(NAMES, masked_every=3)
    ref = _eager_poses(searches, NAMES, pairs)
    r = fmbym.Ragged([searches[k] for k in SIZES], pairs)
    for rep in range(3):
        r.pose.fill_(float("nan"))
        pose = r.launch().clone()
        torch.cuda.synchronize()
        print(f"replay {rep}: max |diff| {torch.nan_to_num(pose - ref, nan=1e9).abs().max().item()}",
              flush=True)
        assert torch.equal(pose, ref), rep
        # eager work between replays
        _ = _eager_poses(searches, NAMES[:2], pairs[:2])
        torch.cuda.synchronize()
    r.close()


def test_ragged_reads_the_scans_at_each_launch():
    searches = _searches()
    names = ["pair128", "batch256", "pair128"]
    pairs = _work_list(names)
    r = fmbym.Ragged([searches[k] for k in SIZES], pairs)
    first = r.launch().clone()
    new = _work_list(names, split="test")
    for q, q2 in zip(pairs, new):
        q[0].copy_(q2[0])
        q[1].copy_(q2[1])
    second = r.launch().clone()
    torch.cuda.synchronize()
    assert torch.equal(second, _eager_poses(searches, names, pairs))
    assert not torch.equal(first, second)
    r.close()


def test_ragged_stamps_follow_the_launch():
    searches = _searches()
    names = ["pair128"] * 6 + ["batch512"] * 2
    pairs = _work_list(names)
    r = fmbym.Ragged([searches[k] for k in SIZES], pairs)
    r.launch()
    torch.cuda.synchronize()
    lat = r.latencies_us()
    print("latencies us", lat.tolist(), flush=True)
    assert fmbym.wall_clock_khz() > 0
    assert bool((lat > 0).all()) and bool((lat < 5e6).all())
    # pairs of one group share the stamp kernel; the small group is not behind the large one
    assert lat[:6].max() <= lat[6:].max()
    r.close()


def test_ragged_pair_against_the_oracle():
    searches = _searches()
    names = ["batch256", "pair128"]
    pairs = _work_list(names)
    r = fmbym.Ragged([searches[k] for k in SIZES], pairs)
    pose = r.launch().cpu().double().numpy()
    for i, name in enumerate(names):
        kw = workloads.search_kwargs(name)
        res = O.search(pairs[i][0].cpu().double().numpy(), pairs[i][1].cpu().double().numpy(),
                       O.Params(**kw))
        ref = np.asarray(res["pose"], dtype=np.float64)
        assert abs(pose[i, 0] - ref[0]) <= 1e-3
        assert np.abs(pose[i, 1:] - ref[1:]).max() <= 1e-3 * kw["delta_xy"]
    r.close()


def test_ragged_network_masks_equal_the_eager_chain():
    """Pairs flagged for network masks: the mask network (inference mode) runs
    inside the launch and the search uses its masks; the pose equals the eager
    MaskNet forward + masked search bit for bit, next to unmasked pairs."""
    from paper_2203_00459_amd.train import he_init
    searches = _searches()
    net = fmbym.MaskNet(he_init(4, 8, seed=4), levels=4)
    nbn = net.bn_running.numel() // 2
    rng = np.random.Generator(np.random.PCG64(8))
    net.bn_running.copy_(torch.tensor(np.concatenate([rng.normal(0, 0.3, nbn), rng.uniform(0.5, 2, nbn)]),
                                      dtype=torch.float32))
    names = ["pair128", "batch256", "pair128", "batch512", "pair128", "batch256"]
    base = _work_list(names)
    pairs = [(q[0], q[1], "net") if i % 2 == 0 else (q[0], q[1]) for i, q in enumerate(base)]
    r = fmbym.Ragged([searches[k] for k in SIZES], pairs, net=net)
    for rep in range(2):
        pose = r.launch().clone()
        torch.cuda.synchronize()
        ref = torch.empty_like(pose)
        for i, (name, q) in enumerate(zip(names, base)):
            s = searches[name]
            if i % 2 == 0:
                m = net.forward(torch.stack([q[0], q[1]]), training=False)
                ref[i] = s.forward(q[0][None], q[1][None], m[0:1].contiguous(), m[1:2].contiguous(),
                                   surfaces=False)["pose"][0]
            else:
                ref[i] = s.forward(q[0][None], q[1][None], surfaces=False)["pose"][0]
        torch.cuda.synchronize()
        print(f"net-masked ragged replay {rep}: max |diff| {(pose - ref).abs().max().item()}", flush=True)
        assert torch.equal(pose, ref)
    r.close()


def test_ragged_rejects_a_size_without_a_plan():
    searches = _searches()
    pairs = _work_list(["pair128", "batch256"])
    with pytest.raises(fmbym.FmbymError):
        fmbym.Ragged([searches["pair128"]], pairs)


def test_one_call_ragged_search_equals_the_launch_object():
    """fmbym_search_ragged (no launch object, no graph): the same poses as the
    captured launch, bit for bit, for a list with unmasked, caller-masked and
    network-masked pairs of the three sizes; twice, the second on a shorter list."""
    from paper_2203_00459_amd.train import he_init
    searches = _searches()
    net = fmbym.MaskNet(he_init(4, 8, seed=6), levels=4)
    base = _work_list(NAMES, masked_every=3)
    pairs = [(q[0], q[1], "net") if i % 4 == 1 else tuple(q) for i, q in enumerate(base)]
    for rep, sub in enumerate((pairs, pairs[2:7])):
        r = fmbym.Ragged([searches[k] for k in SIZES], sub, net=net)
        ref = r.launch().clone()
        pose, st = fmbym.ragged_search([searches[k] for k in SIZES], sub, net=net, stamps=True)
        torch.cuda.synchronize()
        print(f"one-call ragged {rep} ({len(sub)} pairs): max |diff| {(pose - ref).abs().max().item()}",
              flush=True)
        assert torch.equal(pose, ref)
        lat = (st[:-1] - st[-1]).double()
        assert bool((lat > 0).all())
        r.close()
