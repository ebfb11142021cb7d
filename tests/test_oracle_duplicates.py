"""Pins of the oracle's duplicate-track removal: a hand-worked example of
the rule (threshold, ranking, ties), invariance under reordering, and on a
simulated event seeded from every triplet, one kept track per particle.
CPU only."""
import numpy as np

from oracle import oracle as O
from synth import SeedingConfig, generate_event, small_barrel


def test_hand_worked_example():
    A = [1, 2, 3, 4, 5, 6, 7, 8]
    sets = [A,                            # 0: 8 hits, chi2 10
            [1, 2, 3, 4, 5, 9, 10],        # 1: shares 5 of its 7 with 0: duplicate
            [20, 21, 22, 4, 5, 6],         # 2: shares 3 of 6 (exactly half): duplicate
            [30, 31, 32, 7, 8],            # 3: shares 2 of 5 (< half): kept
            list(A),                       # 4: same hits as 0, larger chi2: duplicate
            list(A),                       # 5: same hits and chi2 as 0, smaller seed: ranks first
            [40, 41, 30, 31, 32]]          # 6: shares 3 of 5 with 3, as many hits, larger
    #                                        chi2: a duplicate of 3
    chi2 = [10.0, 1.0, 1.0, 1.0, 12.0, 10.0, 2.0]
    seeds = [[1, 2, 3], [1, 2, 3], [20, 21, 22], [30, 31, 32], [1, 2, 4], [0, 2, 3],
             [40, 41, 42]]
    dup, frag = O.duplicates(sets, chi2, seeds)
    assert list(dup) == [True, True, True, False, True, False, True]
    # 0 and 5 tie on hits and chi2: their order rests on the tie-break
    assert frag[0] and frag[5]
    assert not frag[1] and not frag[3]


def test_flags_do_not_depend_on_track_order():
    rng = np.random.default_rng(51)
    sets, chi2, seeds = [], [], []
    for i in range(60):
        base = rng.integers(0, 40)
        n = rng.integers(4, 10)
        sets.append(sorted(set((base + rng.integers(0, 12, n)).tolist())))
        chi2.append(float(rng.integers(0, 5)))  # ties on purpose
        seeds.append(sorted(rng.choice(100, 3, replace=False).tolist()))
    dup, _ = O.duplicates(sets, chi2, seeds)
    perm = rng.permutation(60)
    dup2, _ = O.duplicates([sets[i] for i in perm], [chi2[i] for i in perm],
                           [seeds[i] for i in perm])
    assert np.array_equal(dup2, dup[perm])


def test_one_kept_track_per_particle_with_triplet_seeds():
    """Small barrel event (no material, no noise) seeded from every triplet:
    among the tracks that hold most of a particle's hits exactly one is
    kept, and no two kept tracks share half of their hits."""
    w = small_barrel()
    ev = generate_event(w, 2)
    trip, _, _ = O.triplet_seeds(w.find, SeedingConfig(), ev)
    res = O.find_event(w.find, w.layers, ev, seeds=trip)
    sets = O.track_hit_sets(res, trip)
    dup, frag = O.duplicates(sets, [r["chi2"] for r in res], trip)
    assert len(res) > 200 and dup.sum() > 0
    owner = {}
    for t, hits in enumerate(ev.track_hits):
        for h in hits:
            owner[h] = t
    kept_per_particle = {}
    for i, s in enumerate(sets):
        if not s:
            continue
        ids, cnt = np.unique([owner[h] for h in s], return_counts=True)
        if cnt.max() >= 0.75 * len(s) and not dup[i]:
            kept_per_particle[ids[cnt.argmax()]] = kept_per_particle.get(ids[cnt.argmax()], 0) + 1
    assert len(kept_per_particle) >= 195
    assert all(v == 1 for v in kept_per_particle.values())
    kept = [set(s) for s, d in zip(sets, dup) if s and not d]
    for i in range(len(kept)):
        for j in range(i + 1, len(kept)):
            assert len(kept[i] & kept[j]) < 0.5 * min(len(kept[i]), len(kept[j]))
