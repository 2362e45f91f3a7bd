"""The C ABI's chain bookkeeping and error paths on the device.

* Chains are independent Markov chains (Hybrid METTS-Ancilla subsection),
  so a batch split over contexts with matching global chain offsets, or a
  chain resumed at sample n from the outcomes of sample n - 1, must
  reproduce the uninterrupted batch bit for bit (every Philox counter
  carries the global chain id and the sample index).
* An evolution applied in parts equals the whole evolution bit for bit.
* The same holds on a U(1) context, with every collapse in S^z.
* The `what` mask of hmps_measure selects outputs without changing them.
* A Jacobi SVD that cannot converge within max_sweeps returns E_NUMERIC and
  poisons the context (E_STATE afterwards); the kernels still exit
  normally, the sweep cap is a host-side limit.
"""
import numpy as np
import pytest

from oracle import hybrid, model
from paper_1910_09142_amd import hmps, workloads

pytestmark = pytest.mark.gpu

# 2x3 ladder, W=1, beta=1, tau=0.1, chi_max=32, cutoff 1e-12
L, W, BETA, TAU, CHI, CUT = 3, 1, 1.0, 0.1, 32, 1e-12


def make(n_chains, **kw):
    n, bonds, order, mask = workloads.ladder_arrays(L, 1.0, 1.0, W)
    lat = hmps.Lattice(n, bonds, order, mask)
    ctx = hmps.Context(n_chains, workloads.mps_length(L, W), CHI, len(bonds),
                       **kw)
    return ctx, lat


def run(ctx, n_samples, first_sample=0):
    out = []
    for n in range(first_sample, first_sample + n_samples):
        ctx.hmps_evolve(BETA, TAU, CHI, CUT)
        m = ctx.hmps_measure()
        m["outcomes"] = ctx.hmps_collapse_resample(n % 2)
        out.append(m)
    return out


def same(a, b, rows=slice(None)):
    for key in ("energy", "bond_ss", "logw", "qn", "outcomes"):
        assert np.array_equal(a[key][rows], b[key]), key


def test_chain_offsets_split_a_batch_bit_for_bit():
    print("case: 4 chains vs 2 + 2 with offsets 0 and 2, seed 11", flush=True)
    ctx, lat = make(4)
    ctx.hmps_init_cluster_env(lat, 4, 11)
    whole = run(ctx, 3)
    ctx.hmps_destroy()
    for off in (0, 2):
        ctx, lat = make(2)
        ctx.hmps_init_cluster_env(lat, 2, 11, chain_offset=off)
        part = run(ctx, 3)
        ctx.hmps_destroy()
        for n in range(3):
            same(whole[n], part[n], slice(off, off + 2))
    # the oracle's chain 3 (global id 3) agrees with the batch's chain 3
    olat = model.ladder(L, 1.0, 1.0, W=W)
    ref = hybrid.run_chain(olat, BETA, TAU, CHI, CUT, 3, seed=11, chain=3)
    lay = model.layout(olat)
    for n in range(3):
        assert abs(whole[n]["energy"][3] - ref[n]["energy"]) <= \
            1e-10 * abs(ref[n]["energy"])
        want = [ref[n]["outcomes"][p] for p in lay.env_positions]
        assert list(whole[n]["outcomes"][3]) == want or ref[n]["near"] > 0
    # distinct chains of one seed are distinct
    assert not np.array_equal(whole[0]["outcomes"][0], whole[0]["outcomes"][1])


def test_resume_at_a_sample_bit_for_bit():
    print("case: 4 samples vs resume at sample 2", flush=True)
    ctx, lat = make(2)
    ctx.hmps_init_cluster_env(lat, 2, 3, chain_offset=5)
    whole = run(ctx, 4)
    ctx.hmps_destroy()
    ctx, lat = make(2)
    # sample 1 collapsed in S^x (odd): its outcomes are the S^x labels
    ctx.hmps_init_cluster_env(lat, 2, 3, env_state=whole[1]["outcomes"],
                              basis=1, chain_offset=5, sample=2)
    assert ctx.hmps_stats().sample == 2
    part = run(ctx, 2, first_sample=2)
    assert ctx.hmps_stats().sample == 4
    ctx.hmps_destroy()
    for n in range(2):
        same(whole[2 + n], part[n])


def test_evolution_in_parts_equals_the_whole():
    print("case: evolve in parts", flush=True)
    env = np.array([[0, 2, 1, 1]], np.uint8)
    ctx, lat = make(1)
    ctx.hmps_init_cluster_env(lat, 1, 0, env_state=env)
    ctx.hmps_evolve(BETA, TAU, CHI, CUT)
    ref = ctx.hmps_measure()
    ns, steps = hmps.hmps_schedule(lat)
    total = 5 * len(steps)
    ctx.hmps_init_cluster_env(lat, 1, 0, env_state=env)
    ctx.hmps_evolve_updates(BETA, TAU, CHI, CUT, 0, 101)
    assert ctx.hmps_stats().evolve_pos == 101
    rank, sig = ctx.hmps_last_spectrum(CHI)
    chi = ctx.hmps_bond_dims()[0]
    k = steps[100 % len(steps)][0]          # update 100 was the last
    assert rank[0] == chi[k + 1] and np.all(np.diff(sig[0, :rank[0]]) <= 0)
    # out of order, changed parameters, or a whole evolution in between
    for bad, code in [((0, 1), hmps.HMPS_E_STATE),
                      ((102, 1), hmps.HMPS_E_STATE),
                      ((101, total), hmps.HMPS_E_INVALID)]:
        with pytest.raises(hmps.HmpsError) as e:
            ctx.hmps_evolve_updates(BETA, TAU, CHI, CUT, *bad)
        assert e.value.status == code
    with pytest.raises(hmps.HmpsError) as e:
        ctx.hmps_evolve_updates(BETA, TAU, CHI, 1e-10, 101, 1)
    assert e.value.status == hmps.HMPS_E_INVALID
    with pytest.raises(hmps.HmpsError) as e:
        ctx.hmps_evolve(BETA, TAU, CHI, CUT)
    assert e.value.status == hmps.HMPS_E_STATE
    # a measurement in the middle leaves the rest of the evolution intact
    ctx.hmps_measure(hmps.MEASURE_LOGW)
    ctx.hmps_evolve_updates(BETA, TAU, CHI, CUT, 101, 1)
    ctx.hmps_evolve_updates(BETA, TAU, CHI, CUT, 102, total - 102)
    assert ctx.hmps_stats().evolve_pos == 0
    assert ctx.hmps_stats().center == 0
    got = ctx.hmps_measure()
    ctx.hmps_destroy()
    for key in ("energy", "bond_ss", "logw", "qn"):
        assert np.array_equal(got[key], ref[key]), key


def test_measure_mask_selects_outputs():
    print("case: measure mask", flush=True)
    ctx, lat = make(2)
    ctx.hmps_init_cluster_env(lat, 2, 4)
    ctx.hmps_evolve(BETA, TAU, CHI, CUT)
    full = ctx.hmps_measure()
    for what, keys in [(hmps.MEASURE_LOGW, ["logw"]),
                       (hmps.MEASURE_QN, ["qn"]),
                       (hmps.MEASURE_BONDS | hmps.MEASURE_LOGW,
                        ["bond_ss", "logw"]),
                       (hmps.MEASURE_ENERGY, ["energy"])]:
        part = ctx.hmps_measure(what)
        for key in ("energy", "bond_ss", "logw", "qn"):
            if key in keys:
                assert np.array_equal(part[key], full[key]), key
            else:
                assert part[key] is None
    # accumulating moments is not an output
    acc = ctx.hmps_measure(hmps.MEASURE_ACCUMULATE)
    assert all(v is None for v in acc.values())
    with pytest.raises(hmps.HmpsError) as e:
        ctx.hmps_measure(32)
    assert e.value.status == hmps.HMPS_E_INVALID
    assert np.array_equal(ctx.hmps_measure()["energy"], full["energy"])
    ctx.hmps_destroy()


def test_sweep_cap_gives_numeric_error_then_state_error():
    # the 2x8 ladder reaches 384 x 384 theta' (blocked Jacobi): one sweep
    # can never certify convergence there
    print("case: max_sweeps=1 on the 2x8 ladder", flush=True)
    n, bonds, order, mask = workloads.ladder_arrays(8, 1.0, 1.0, 2)
    lat = hmps.Lattice(n, bonds, order, mask)
    ctx = hmps.Context(1, workloads.mps_length(8, 2), 128, len(bonds),
                       max_sweeps=1)
    ctx.hmps_init_cluster_env(lat, 1, 0)
    with pytest.raises(hmps.HmpsError) as e:
        ctx.hmps_evolve(1.0, 0.05, 128, 1e-12)
    assert e.value.status == hmps.HMPS_E_NUMERIC
    assert "converge" in str(e.value)
    for call in (lambda: ctx.hmps_measure(),
                 lambda: ctx.hmps_evolve(1.0, 0.05, 128, 1e-12),
                 lambda: ctx.hmps_collapse_resample(0),
                 lambda: ctx.hmps_init_cluster_env(lat, 1, 0)):
        with pytest.raises(hmps.HmpsError) as e:
            call()
        assert e.value.status == hmps.HMPS_E_STATE
    s = ctx.hmps_stats()
    assert s.updates > 0
    ctx.hmps_destroy()


def test_split_bf16_precision_is_rejected():
    with pytest.raises(hmps.HmpsError) as e:
        make(1, precision=hmps.PREC_MIXED_BF16X3)
    assert e.value.status == hmps.HMPS_E_INVALID


def run_z(ctx, n_samples):
    out = []
    for _ in range(n_samples):
        ctx.hmps_evolve(BETA, TAU, CHI, CUT)
        m = ctx.hmps_measure()
        m["outcomes"] = ctx.hmps_collapse_resample(0)
        out.append(m)
    return out


def test_u1_offsets_resume_and_parts_bit_for_bit():
    # the same bookkeeping on a U(1) context (every collapse in S^z): a
    # split batch, a resumed chain and an evolution in parts reproduce the
    # uninterrupted runs bit for bit
    print("case: U(1) offsets, resume, parts", flush=True)
    u1 = {"symmetry": hmps.SYM_U1}
    ctx, lat = make(4, **u1)
    ctx.hmps_init_cluster_env(lat, 4, 11)
    whole = run_z(ctx, 3)
    ctx.hmps_destroy()
    for off in (0, 2):
        ctx, lat = make(2, **u1)
        ctx.hmps_init_cluster_env(lat, 2, 11, chain_offset=off)
        part = run_z(ctx, 3)
        ctx.hmps_destroy()
        for n in range(3):
            same(whole[n], part[n], slice(off, off + 2))
    # resume at sample 2 from the S^z outcomes of sample 1
    ctx, lat = make(4, **u1)
    ctx.hmps_init_cluster_env(lat, 4, 11, env_state=whole[1]["outcomes"],
                              sample=2)
    part = run_z(ctx, 1)
    ctx.hmps_destroy()
    same(whole[2], part[0])
    # an evolution in parts
    env = np.array([[0, 2, 1, 1]], np.uint8)
    ctx, lat = make(1, **u1)
    ctx.hmps_init_cluster_env(lat, 1, 0, env_state=env)
    ctx.hmps_evolve(BETA, TAU, CHI, CUT)
    ref = ctx.hmps_measure()
    ns, steps = hmps.hmps_schedule(lat)
    total = 5 * len(steps)
    ctx.hmps_init_cluster_env(lat, 1, 0, env_state=env)
    for first, count in ((0, 37), (37, 64), (101, total - 101)):
        ctx.hmps_evolve_updates(BETA, TAU, CHI, CUT, first, count)
    got = ctx.hmps_measure()
    ctx.hmps_destroy()
    for key in ("energy", "bond_ss", "logw", "qn"):
        assert np.array_equal(got[key], ref[key]), key
