"""Per-kernel timing (hp_profile_enable / hp_profile_read): launch counts are exact, the kernel
filter holds, and launches from threads iterating their own contexts at the same time are all
counted (the profiler state is process-wide and guarded)."""
import threading

import pytest

from paper_2402_18311_amd import netgen

pytestmark = pytest.mark.gpu


def test_profiler_counts_launches_from_concurrent_threads():
    import torch

    from paper_2402_18311_amd import hybro as hy
    nl = netgen.make_netlist("tiny", 0)
    gamma = 4 * nl.bin_w
    pls = [hy.Placer(nl, precision=64, stream=torch.cuda.Stream()) for _ in range(2)]
    try:
        slots = []
        for pl in pls:
            s = pl.new_slot()
            pl.set_positions(s, nl.x0, nl.y0)
            pl.iterate(s, gamma, 2, hpwl=False)
            slots.append(s)
        torch.cuda.synchronize()
        hy.hp_profile_enable(pls[0].ctx, True, "eval_front_kernel")
        hy.hp_profile_read(pls[0].ctx, reset=True)
        ths = [threading.Thread(target=pl.iterate, args=(s, gamma, 25), kwargs={"hpwl": False})
               for pl, s in zip(pls, slots)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        prof = hy.hp_profile_read(pls[0].ctx, reset=True)
        assert set(prof) == {"eval_front_kernel"} and prof["eval_front_kernel"][0] == 50
        assert prof["eval_front_kernel"][1] > 0
        # every kernel: one update per iteration
        hy.hp_profile_enable(pls[0].ctx, True)
        pls[1].iterate(slots[1], gamma, 3, hpwl=False)
        prof = hy.hp_profile_read(pls[1].ctx, reset=True)
        assert prof["step_update_kernel"][0] == 3 and prof["eval_front_kernel"][0] == 3
    finally:
        for pl in pls:
            hy.hp_profile_enable(pl.ctx, False)
            pl.close()
