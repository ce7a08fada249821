"""Precision policy at full size: the 1024x512 N_H = 4 airfoil iterated in
FP32 bulk and in FP64 (batched) for N iterations (default 60000), residual
drop printed every 10000, then the relative 2-norm difference of the force
harmonics (cl, cd, cm).  Run on one GPU:
    python tests/run_precision_full_size.py [N]
"""
import os, sys, time, torch
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import hb_oracle as O
from paper_1304_7654_amd import hb, synth
N = int(sys.argv[1]) if len(sys.argv) > 1 else 60000
chunk = 10000
p = synth.make_problem("naca1024x512_nh4")
p.solver.graph_iters = 50
q0 = torch.as_tensor(synth.initial_state(p)).to("cuda")
res = {}
for prec in (1, 0):
    g = hb.Grid(p.blocks, p.flow, p.solver, precision=prec, batched=1)
    if prec == 1:
        g.autotune(q0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1304_7654_amd", "tune_cache.json"))
    q = q0.clone()
    norms = torch.zeros(N, dtype=torch.float64, device="cuda")
    cf = torch.zeros(g.n_forces, dtype=torch.float64, device="cuda")
    t = time.time()
    first = None
    for k in range(0, N, chunk):
        g.rk_iterate(q, chunk, norms[k:k + chunk], cf)
        torch.cuda.synchronize()
        n = norms.cpu()
        first = float(n[0])
        print("prec", prec, "it", k + chunk, "drop %.3e" % (float(n[k + chunk - 1]) / first), "t %.0f s" % (time.time() - t), "status", g.status(), flush=True)
    c = cf.cpu().reshape(-1, 9, 3)[0]
    res[prec] = ([O.harmonics(c[:, j]) for j in range(3)], float(norms[-1].item()) / first)
    g.close()
for j, nm in enumerate(("cl", "cd", "cm")):
    h64, h32 = res[0][0][j], res[1][0][j]
    print("RESULT %s FP64 harmonics %s rel err FP32 %.3e" % (nm, [round(float(x), 6) for x in h64], float((h32 - h64).norm() / h64.norm())), flush=True)
print("RESULT drops FP64 %.3e FP32 %.3e" % (res[0][1], res[1][1]), flush=True)
