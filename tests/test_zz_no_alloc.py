"""lst_run_event_noalloc (no device allocation: intermediate buffers in the
library's static workspace, outputs in caller-owned device buffers) against
lst_run_event, through the C ABI: two calls in a row, the second on a smaller
event, give exactly the lists of the allocating entry point."""
import numpy as np
import pytest

from paper_2407_18231_amd import lst, synth as s
from parity import STAGES

pytestmark = pytest.mark.gpu

CAPS = dict(md=100_000, ls=600_000, t3=400_000, t5=100_000, pt3=60_000, pt5=30_000, tc=60_000)


def _dev(ev, torch):
    d = {k: torch.from_numpy(np.ascontiguousarray(ev[k])).to("cuda:0")
         for k in ("x", "y", "z", "pls_par", "pls_cov", "sensor")}
    d["module"] = torch.from_numpy(ev["module"].astype(np.int32)).to("cuda:0")
    return d


def test_noalloc_matches_run_event():
    torch = pytest.importorskip("torch")
    g = s.make_geometry("pu200")
    big = s.gen_event(g, s.config_pu(250), s.event_seed(2, 50))
    small = s.gen_event(g, s.config_pu(60), s.event_seed(2, 51))
    with lst.Context() as c:
        c.load_geometry(g)
        bufs = {k: torch.full((n, 2), -1, dtype=torch.int32, device="cuda:0") for k, n in CAPS.items()}
        kap = torch.zeros(CAPS["t3"], dtype=torch.float32, device="cuda:0")
        stream = torch.cuda.Stream()
        for ev in (big, small):
            ref = c.run_event(ev)
            dev = _dev(ev, torch)
            torch.cuda.synchronize()
            n = c.run_event_noalloc(dev, bufs, kap, stream)
            print({k: n[k] for k in STAGES}, flush=True)
            for k in STAGES:
                assert n[k] == len(ref[k]), k
                got = bufs[k][:n[k]].cpu().numpy().view(np.uint32)
                assert np.array_equal(got, ref[k]), k
            assert np.array_equal(kap[:n["t3"]].cpu().numpy().view(np.uint32), ref["t3_kappa"].view(np.uint32))
            assert len(ref["pt5"]) > 0 and n["ls"] > 5_000


def test_noalloc_errors():
    torch = pytest.importorskip("torch")
    g = s.make_geometry("pu200")
    ev = s.gen_event(g, s.config_pu(80), s.event_seed(2, 52))
    with lst.Context() as c:
        c.load_geometry(g)
        ref = c.run_event(ev)
        dev = _dev(ev, torch)
        torch.cuda.synchronize()
        # output buffers below the event's counts: TOO_LARGE, counts reported
        small = {k: torch.zeros((4, 2), dtype=torch.int32, device="cuda:0") for k in STAGES}
        with pytest.raises(lst.LstError) as e:
            c.run_event_noalloc(dev, small)
        assert e.value.name == "TOO_LARGE"
        assert e.value.counts["ls"] == len(ref["ls"])
        # host pointers are refused
        bufs = {k: torch.zeros((n, 2), dtype=torch.int32, device="cuda:0") for k, n in CAPS.items()}
        with pytest.raises(lst.LstError) as e:
            c.run_event_noalloc(ev, bufs)
        assert e.value.name == "INVALID_ARG"
        # more hits than the workspace's limit
        many = {k: torch.cat([dev[k]] * 7) for k in ("x", "y", "z", "module", "sensor")}
        many.update(pls_par=dev["pls_par"], pls_cov=dev["pls_cov"])
        assert many["x"].numel() > lst.NOALLOC_MAX_HITS
        with pytest.raises(lst.LstError) as e:
            c.run_event_noalloc(many, bufs)
        assert e.value.name == "TOO_LARGE"
        # and the entry point still works afterwards
        n = c.run_event_noalloc(dev, bufs)
        for k in STAGES:
            assert np.array_equal(bufs[k][:n[k]].cpu().numpy().view(np.uint32), ref[k]), k
