"""Shared check of the reporter outputs (speciation events, species abundance)
against the species ids a run produced and, optionally, the oracle."""
import numpy as np

import oracle


def check_reporters(species, rich, rep, seed, osc=None, samples=None):
    """The speciation event behind every sample names its species; the abundance pairs are the
    species ids with their sample counts; optionally the event times equal the oracle's."""
    loc = rep["spec_loc"].cpu().numpy().view(np.uint32)
    tm = rep["spec_time"].cpu().numpy()
    for q in range(len(species)):
        assert oracle.species_id(seed, int(loc[q]), float(tm[q])) == int(species[q])
    ids = rep["abundance_ids"].cpu().numpy().view(np.uint64)[:rich]
    cnt = rep["abundance_counts"].cpu().numpy()[:rich]
    u, c = np.unique(species, return_counts=True)
    order = np.argsort(ids)
    assert np.array_equal(ids[order], u) and np.array_equal(cnt[order], c)
    if osc is not None:
        _, ts, _ = osc.simulate_naive(seed, samples)
        assert np.array_equal(tm, ts)
