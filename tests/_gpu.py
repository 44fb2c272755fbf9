"""Helpers for the GPU tests: run libjefi through its C ABI on torch device
memory and return numpy results."""
import numpy as np

PREC = {"f64": (1, 0), "f32": (0, 1)}  # name -> (history dtype, precision)


def gpu_eval(p, prec="f32", out_dtype=None, obs=None, capacity=None, screen=None, c=None, tile=0, flags=0):
    import torch
    import paper_2104_05426_amd as J
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    pr = J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP
    obs = obs or p.obs
    store, h = J.upload_history(p.src, p.hist, hdt, t0=p.t0, newest=p.newest, capacity=capacity)
    tdt = torch.float64 if (out_dtype or prec) == "f64" else torch.float32
    n = obs.size
    E = torch.full((3, max(n, 1)), float("nan"), dtype=tdt, device="cuda")
    B = torch.full((3, max(n, 1)), float("nan"), dtype=tdt, device="cuda")
    opt = J.jefi_options_default(precision=pr, c=c if c is not None else p.c,
                                 screen=screen if screen is not None else p.screen)
    opt.tile_config = tile
    opt.flags = flags
    J.jefi_eval_fields(p.src, h, p.dt, p.nt, obs, p.t, E[:, :n] if n else E, B[:, :n] if n else B, opt)
    torch.cuda.synchronize()
    out = E[:, :n].double().cpu().numpy(), B[:, :n].double().cpu().numpy()
    del store
    return out


def gpu_fingerprint(p, prec="f32", tile=0, flags=0):
    import torch
    import paper_2104_05426_amd as J
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    pr = J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP
    store, h = J.upload_history(p.src, p.hist, hdt, t0=p.t0, newest=p.newest)
    fp = torch.zeros((p.obs.size, 4), dtype=torch.int64, device="cuda")
    opt = J.jefi_options_default(precision=pr, c=p.c, screen=p.screen)
    opt.tile_config = tile
    opt.flags = flags
    J.jefi_slice_fingerprint(p.src, h, p.dt, p.nt, p.obs, p.t, fp, opt)
    torch.cuda.synchronize()
    out = fp.cpu().numpy()
    del store
    return out


def gpu_dump(p, prec="f32"):
    import torch
    import paper_2104_05426_amd as J
    pr = J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP
    out = torch.zeros((p.obs.size, p.src.size), dtype=torch.int32, device="cuda")
    opt = J.jefi_options_default(precision=pr, c=p.c, screen=p.screen)
    J.jefi_slice_index_dump(p.src, p.nt, p.dt, p.newest, p.t0, p.obs, p.t, out, opt)
    torch.cuda.synchronize()
    return out.cpu().numpy()


class BatchRun:
    """Histories and outputs of a list of problems resident on the GPU, for
    batched and solo evaluation through the C ABI."""

    def __init__(self, problems, prec="f32"):
        import torch
        import paper_2104_05426_amd as J
        self.J = J
        self.problems = problems
        self.prec = prec
        hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
        self.tdt = torch.float64 if prec == "f64" else torch.float32
        self.stores, self.hists, self.E, self.B = [], [], [], []
        for p in problems:
            st, h = J.upload_history(p.src, p.hist, hdt, t0=p.t0, newest=p.newest)
            self.stores.append(st)
            self.hists.append(h)
            n = max(p.obs.size, 1)
            self.E.append(torch.full((3, n), float("nan"), dtype=self.tdt, device="cuda"))
            self.B.append(torch.full((3, n), float("nan"), dtype=self.tdt, device="cuda"))

    def options(self, tile=0, flags=0, reserve_cus=0):
        J = self.J
        pr = J.JEFI_PREC_F64 if self.prec == "f64" else J.JEFI_PREC_F32_COMP
        opt = J.jefi_options_default(precision=pr)
        opt.tile_config = tile
        opt.flags = flags
        opt.reserve_cus = reserve_cus
        return opt

    def problem_structs(self):
        J = self.J
        return [J.make_problem(p.src, h, p.dt, p.nt, p.obs, p.t, E, B)
                for p, h, E, B in zip(self.problems, self.hists, self.E, self.B)]

    def run_batch(self, tile=0, flags=0, reserve_cus=0):
        import torch
        for E, B in zip(self.E, self.B):
            E.fill_(float("nan"))
            B.fill_(float("nan"))
        self.J.jefi_eval_batch(self.problem_structs(), self.options(tile, flags, reserve_cus))
        torch.cuda.synchronize()
        return self.results()

    def run_solo(self, tile=0, flags=0):
        import torch
        for p, h, E, B in zip(self.problems, self.hists, self.E, self.B):
            E.fill_(float("nan"))
            B.fill_(float("nan"))
            self.J.jefi_eval_fields(p.src, h, p.dt, p.nt, p.obs, p.t, E, B, self.options(tile, flags))
        torch.cuda.synchronize()
        return self.results()

    def results(self):
        return [(E[:, :p.obs.size].double().cpu().numpy(), B[:, :p.obs.size].double().cpu().numpy())
                for p, E, B in zip(self.problems, self.E, self.B)]
