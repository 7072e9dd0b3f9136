"""Precision studies of the storage formats on the GPU.

The FP64 storage path (parity-proven against the FP64 CPU oracle) is the
reference; FP32, FP16-shifted and BF16-shifted storage are compared with it on
the rising bubble (rise velocity, centroid, mass, interface width over time)
and on the bubble swarm (phase field after N steps, mass drift).

    python -m paper_2012_06144_amd.studies rising --steps 20000 --out rising.json
    python -m paper_2012_06144_amd.studies swarm --steps 2000 --out swarm.json

The drag study (Sec. 6.1): the single rising bubble at Eo = 30 for several
gravity Reynolds numbers; the terminal velocity gives C_D^LBM, compared with
the Bhaga-Weber correlation.

    python -m paper_2012_06144_amd.studies drag --re 10,20,30,60 --out drag.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

STORAGES = ("f64", "f32", "f16s", "bf16s")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def rising_bubble(steps: int = 20000, every: int = 500, storages=STORAGES, grid=None):
    """Trajectories of the rising bubble (128 x 512 x 128, D = 32, Eo ~ 10)."""
    import torch

    from . import inputs, lbm
    s = inputs.rising_bubble() if grid is None else inputs.rising_bubble(*grid)
    phi, u, ps = inputs.build_fields(s)
    out = {"workload": s.name, "steps": steps, "every": every, "runs": {}}
    for st in storages:
        sv = lbm.Solver(s.physics(), storage=st)
        sv.init_fields(phi, u, ps)
        traj = []
        t0 = time.perf_counter()
        s0 = sv.stats()
        traj.append(dict(step=0, **_pick(s0)))
        for k in range(every, steps + 1, every):
            sv.step(every)
            traj.append(dict(step=k, **_pick(sv.stats())))
        torch.cuda.synchronize()
        out["runs"][st] = {"trajectory": traj, "seconds": time.perf_counter() - t0}
        _log(f"[rising] {st}: y_c {traj[-1]['centroid_y']:.3f} U {traj[-1]['rise_velocity']:.4e} "
             f"mass drift {(traj[-1]['mass'] - traj[0]['mass']) / traj[0]['mass']:.2e}")
        del sv
        torch.cuda.empty_cache()
    _summarise_rising(out)
    return out


def _pick(st):
    return {"centroid_y": st["centroid"][1], "rise_velocity": st["rise_velocity"], "mass": st["mass"],
            "xi_eff": st["xi_eff"], "max_speed": st["max_speed"], "gas_volume": st["gas_volume"]}


def _summarise_rising(out):
    ref = out["runs"]["f64"]["trajectory"] if "f64" in out["runs"] else None
    summary = {}
    for st, run in out["runs"].items():
        tr = run["trajectory"]
        d = {"mass_drift_rel": (tr[-1]["mass"] - tr[0]["mass"]) / tr[0]["mass"],
             "final_rise_velocity": tr[-1]["rise_velocity"], "final_centroid_y": tr[-1]["centroid_y"],
             "final_xi_eff": tr[-1]["xi_eff"]}
        if ref is not None:
            # error over the second half of the run, where the bubble rises steadily
            half = len(tr) // 2
            uref = np.array([r["rise_velocity"] for r in ref[half:]])
            uu = np.array([r["rise_velocity"] for r in tr[half:]])
            yref = np.array([r["centroid_y"] for r in ref])
            yy = np.array([r["centroid_y"] for r in tr])
            d["rise_velocity_rel_err_max"] = float(np.max(np.abs(uu - uref)) / np.max(np.abs(uref)))
            d["rise_velocity_rel_err_final"] = float(abs(uu[-1] - uref[-1]) / abs(uref[-1]))
            rise = yref[-1] - yref[0]
            d["centroid_err_max_cells"] = float(np.max(np.abs(yy - yref)))
            d["centroid_err_rel_to_rise"] = float(np.max(np.abs(yy - yref)) / abs(rise)) if rise else None
        summary[st] = d
    out["summary"] = summary


def swarm(steps: int = 2000, storages=STORAGES, n: int = 512):
    """Phase field and mass of the bubble swarm after ``steps`` steps."""
    import torch

    from . import inputs, lbm
    s = inputs.bubble_swarm(n=n)
    phi, u, ps = inputs.build_fields(s)
    fluid = s.nx * s.nz * (s.ny - 2)
    out = {"workload": s.name, "steps": steps, "runs": {}}
    ref_phi = None
    for st in storages:
        sv = lbm.Solver(s.physics(), storage=st)
        sv.init_fields(phi, u, ps)
        m0 = sv.reduce_mass()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        try:
            stt = sv.stats()
        except lbm.LbmError as e:
            first_bad = _first_nonfinite_step(s, phi, u, ps, st, steps)
            out["runs"][st] = {"finite": False, "first_nonfinite_step": first_bad, "error": str(e),
                               "seconds": dt, "mlups": fluid * steps / dt / 1e6}
            _log(f"[swarm] {st}: NOT FINITE (first non-finite statistics at step {first_bad}); "
                 f"{fluid * steps / dt / 1e6:.0f} MLUPS")
            del sv
            torch.cuda.empty_cache()
            continue
        ph, _, _ = sv.macroscopic(torch.float32)
        ph = ph.cpu().numpy().astype(np.float64)
        r = {"mass_drift_rel": (stt["mass"] - m0) / m0, "seconds": dt, "mlups": fluid * steps / dt / 1e6,
             "gas_volume": stt["gas_volume"], "xi_eff": stt["xi_eff"], "max_speed": stt["max_speed"],
             "rise_velocity": stt["rise_velocity"], "finite": bool(np.isfinite(ph).all())}
        if st == "f64":
            ref_phi = ph
        elif ref_phi is not None:
            d = ph - ref_phi
            r["phi_err_max"] = float(np.abs(d).max())
            r["phi_err_rms"] = float(np.sqrt(np.mean(d * d)))
        out["runs"][st] = r
        _log(f"[swarm] {st}: {r['mlups']:.0f} MLUPS, mass drift {r['mass_drift_rel']:.2e}, "
             f"phi err max {r.get('phi_err_max', 0):.2e}")
        del sv, ph
        torch.cuda.empty_cache()
    return out


def _first_nonfinite_step(s, phi, u, ps, st, steps, chunk=100):
    """Reruns the case in chunks and returns the first step count after which
    the statistics are no longer finite (None if it stays finite)."""
    import torch

    from . import lbm
    sv = lbm.Solver(s.physics(), storage=st)
    sv.init_fields(phi, u, ps)
    done = 0
    try:
        while done < steps:
            sv.step(chunk)
            done += chunk
            st_ = sv.stats()
            _log(f"[swarm]   {st} step {done}: max|u| {st_['max_speed']:.3e} xi_eff {st_['xi_eff']:.3f} "
                 f"mass {st_['mass']:.6e}")
        return None
    except lbm.LbmError:
        return done
    finally:
        del sv
        torch.cuda.empty_cache()


def drag_coefficient_lbm(g: float, rho_H: float, rho_L: float, D: float, u_t: float) -> float:
    """C_D from the terminal velocity (Sec. 6.1): 4/3 g (rho_H - rho_L) D / (rho_H u_t^2)."""
    return 4.0 / 3.0 * g * (rho_H - rho_L) * D / (rho_H * u_t * u_t)


def drag_coefficient_bhaga_weber(re: float) -> float:
    """Bhaga and Weber's correlation as printed (eq. analytical_drag_coeff):
    [2.67^(9/10) + (16/Re)^(9/10)]^(10/9)."""
    return (2.67 ** 0.9 + (16.0 / re) ** 0.9) ** (10.0 / 9.0)


def drag(re_list=(10.0, 20.0, 30.0, 60.0), eo: float = 30.0, t_ref: float = 2000.0, t_end: float = 10.0,
         every: int = 500, storage: str = "f32", grid=(256, 1024, 256), D: float = 32.0, lattice=None):
    """Rising bubble at Eo = eo for each gravity Reynolds number: trajectory of
    the gas-weighted rise velocity and centroid to t* = t_end; the terminal
    velocity is the mean rise velocity over t* in [0.8 t_end, t_end]."""
    import torch

    from . import inputs, lbm
    lattice = dict(lattice or {})
    out = {"eo": eo, "t_ref": t_ref, "t_end": t_end, "storage": storage, "grid": list(grid), "D": D,
           "lattice": lattice, "runs": {}}
    for re in re_list:
        s = inputs.drag_bubble(re, eo=eo, D=D, t_ref=t_ref, grid=grid)
        phi, u, ps = inputs.build_fields(s)
        sv = lbm.Solver(dict(s.physics(), **lattice), storage=storage)
        sv.init_fields(phi, u, ps)
        steps = int(round(t_end * t_ref))
        traj = [dict(step=0, **_pick(sv.stats()))]
        t0 = time.perf_counter()
        for k in range(every, steps + 1, every):
            sv.step(every)
            traj.append(dict(step=k, **_pick(sv.stats())))
            if k % (10 * every) == 0:
                _log(f"[drag] Re_Gr {re:g}: step {k}/{steps} t* {k / t_ref:.2f} U {traj[-1]['rise_velocity']:.4e} "
                     f"y_c {traj[-1]['centroid_y']:.1f}")
        torch.cuda.synchronize()
        g = -s.accel[1]
        tail = [r for r in traj if r["step"] >= 0.8 * steps]
        u_t = float(np.mean([r["rise_velocity"] for r in tail]))
        ys = np.array([r["centroid_y"] for r in tail])
        ts = np.array([r["step"] for r in tail], dtype=float)
        u_slope = float(np.polyfit(ts, ys, 1)[0]) if len(ts) > 1 else None
        mu_H = s.rho_H * s.tau_H / 3.0
        re_t = s.rho_H * u_t * D / mu_H
        cd = drag_coefficient_lbm(g, s.rho_H, s.rho_L, D, u_t)
        rec = {"re_gr": re, "g": g, "sigma": s.sigma, "tau_H": s.tau_H, "tau_L": s.tau_L, "steps": steps,
               "seconds": time.perf_counter() - t0, "u_t": u_t, "u_t_centroid_slope": u_slope,
               "re_terminal": re_t, "cd_lbm": cd,
               "cd_bhaga_weber_at_re_gr": drag_coefficient_bhaga_weber(re),
               "cd_bhaga_weber_at_re_terminal": drag_coefficient_bhaga_weber(re_t),
               "mass_drift_rel": (traj[-1]["mass"] - traj[0]["mass"]) / traj[0]["mass"],
               "final_xi_eff": traj[-1]["xi_eff"], "trajectory": traj}
        out["runs"][f"{re:g}"] = rec
        _log(f"[drag] Re_Gr {re:g}: u_t {u_t:.4e} (centroid slope {u_slope:.4e}), Re_t {re_t:.2f}, "
             f"C_D {cd:.3f}; Bhaga-Weber {rec['cd_bhaga_weber_at_re_gr']:.3f} at Re_Gr, "
             f"{rec['cd_bhaga_weber_at_re_terminal']:.3f} at Re_t; {rec['seconds']:.0f} s")
        del sv
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["rising", "swarm", "drag"])
    ap.add_argument("--re", default="10,20,30,60", help="gravity Reynolds numbers of the drag study")
    ap.add_argument("--eo", type=float, default=30.0)
    ap.add_argument("--t-ref", type=float, default=2000.0, help="reference time sqrt(D/g) in steps (drag study)")
    ap.add_argument("--t-end", type=float, default=10.0, help="end of the drag study in units of t_ref")
    ap.add_argument("--lattice", default="15,27,0",
                    help="phase-field set, hydrodynamic set and phase-field MRT (0/1) of the drag study")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--storages", default=",".join(STORAGES))
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    sts = tuple(a.storages.split(","))
    if a.study == "rising":
        res = rising_bubble(a.steps or 20000, a.every, sts)
    elif a.study == "drag":
        qp, qh, mrt = (int(v) for v in a.lattice.split(","))
        res = drag(tuple(float(v) for v in a.re.split(",")), eo=a.eo, t_ref=a.t_ref, t_end=a.t_end,
                   every=a.every, storage=sts[0] if len(sts) == 1 else "f32",
                   lattice=dict(lattice_phase=qp, lattice_hydro=qh, phase_mrt=bool(mrt)))
        res["summary"] = {k: {kk: v for kk, v in r.items() if kk != "trajectory"} for k, r in res["runs"].items()}
    else:
        res = swarm(a.steps or 2000, sts)
    txt = json.dumps(res, indent=1)
    if a.out:
        open(a.out, "w").write(txt)
    print(json.dumps(res.get("summary", {k: v for k, v in res["runs"].items()}), indent=1))


if __name__ == "__main__":
    main()
