"""The allocation-free energy entry point (cw_energy_noalloc, through the C
ABI) against cw_energy: the same kernels with the partial sums in the
library's static scratch instead of the workspace.  Two calls in a row, the
second on a smaller simulation; sizes beyond the scratch are refused."""
import numpy as np
import pytest

from paper_2302_13907_amd import cwell, inputs

from gpu_common import Scenario, announce, run_gpu

pytestmark = pytest.mark.gpu


def _sim(shape, steps, seed):
    med = inputs.cased_well(*shape, 5e-3, 5e-3, z_top=shape[2] * 5e-3 / 2, rock_jitter=0.02, seed=seed)
    sc = Scenario(shape=shape, h=(5e-3, 5e-3), medium=med, steps=steps, npml=(4, 4),
                  sources=[("volume", 0, -1, shape[2] // 3, 1.0)])
    return run_gpu(sc, keep_sim=True)[2]


def test_energy_noalloc_matches_energy():
    sims = []
    for shape, steps, nblocks in (((48, 32, 192), 120, 4096), ((16, 6, 40), 60, 37)):
        announce("energy without allocation on %s after %d steps" % (shape, steps))
        s = _sim(shape, steps, seed=len(sims) + 1)
        ref = s.energy()
        assert ref > 0
        same = s.energy_noalloc(1024)          # cw_energy's block count: bitwise its result
        other = s.energy_noalloc(nblocks)      # another summation order
        announce("  cw_energy %.17g, noalloc(1024) %.17g, noalloc(%d) %.17g" % (ref, same, nblocks, other))
        assert same == ref
        assert abs(other / ref - 1.0) < 1e-12
        sims.append((s, ref))
    # the first simulation again, after the second overwrote the scratch
    s, ref = sims[0]
    assert s.energy_noalloc(1024) == ref
    for bad in (0, -3, 4097):
        with pytest.raises(cwell.CwellError) as e:
            s.energy_noalloc(bad)
        assert e.value.status == -2
    for s, _ in sims:
        s.close()
