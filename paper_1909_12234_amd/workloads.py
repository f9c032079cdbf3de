"""Named synthetic workloads (lattice, gauge recipe, mass, probes, tolerances).

Gauge fields are seeded random SU(3) links U = exp(i eps H), H = sum_a w_a lambda_a with
standard-normal w_a (the `synth` package).  Probes are the real Rademacher probes of the
library (SplitMix64 counter hash) with the seeds below.
"""

WORKLOADS = {
    # 4^4, the small workload: exact trace by dense LU
    "wilson4x4_plain": dict(dims=(4, 4, 4, 4), eps=0.3, seed=1, mass=0.1, nprobes=64, probe_seed=1000,
                            xi=1e-10, k=16, inner_prec="f64"),
    # 16^3x32 mixed precision: FP16 inner s-step cycles (packed half arithmetic in the operator,
    # FP32 accumulation), FP64 defect correction to 1e-8, k = 64 basis.
    # The mass is the most ill-conditioned one at which FP64 GMRES(32) still converges within
    # 5000 steps (kappa(A) = sigma_max / min |lambda(A g5)|, measured for these fields:
    # m = -1.90: 430, -1.92: 740, -1.94: 1.7e3, -1.95: 3.8e3 (about 2800 steps),
    # -1.96: 9.5e3, where restarted GMRES stagnates past 5000 steps).
    # s-step cycles of 15: GMRES steps per probe barely depend on the restart length while the
    # Gram-Schmidt traffic per step grows with it; s-step cycles replace that traffic by one
    # Gram pass per cycle, and longer cycles spread the FP64 restart over more steps.
    "wilson16x32_mixed": dict(dims=(16, 16, 16, 32), eps=0.5, seed=1, mass=-1.95, nprobes=128, probe_seed=1001,
                              xi=1e-8, k=64, inner_prec="f16", restart=15, sstep=1),
    # three lattices solved one after the other in a batch of 192 probes, FP32 storage
    "wilson_batched3": dict(lattices=[((8, 8, 8, 8), 1), ((12, 12, 12, 24), 2), ((16, 16, 16, 32), 3)], eps=0.4,
                            mass=0.1, nprobes=192, probe_seed=1002, xi=1e-8, inner_prec="f32"),
    # 16^3x32 with the learned preconditioner, 256 probes
    # the net is trained before the timed region on 1024 pairs (e = the FP32 solver's output for a
    # Gaussian field at 1e-2, r = A e) in 4 epochs
    "wilson16x32_net": dict(dims=(16, 16, 16, 32), eps=0.5, seed=1, mass=-1.90, nprobes=256, probe_seed=1003,
                            xi=1e-8, inner_prec="bf16", train_pairs=1024, train_epochs=4, pair_xi=1e-2),
    # 32^3x64 prolongator deflation (Algorithm 2): 4^4 aggregates, 24 near-null vectors per
    # chirality (FP16 s-step solves to 1e-2 or 200 steps), explicit coarse operator, k = 256
    # coarse eigenvectors; 256 probes solved 32 at a time with the 16^3x32 workload's solver
    "wilson32x64_mg": dict(dims=(32, 32, 32, 64), eps=0.5, seed=1, mass=-1.90, nprobes=256, probe_seed=1004,
                           xi=1e-8, block=(4, 4, 4, 4), nv=24, k=256, inner_prec="f16", restart=15, sstep=1,
                           batch=32),
    # the same with a second multigrid level (Table 2: 2^4 blocks of the 8^3x16 coarse lattice,
    # 32 near-null vectors of the coarse operator per chirality, nc2 = 32768); the k = 256
    # coarse eigenvectors come from the level-2 operator (Table 3's two-level deflation space)
    "wilson32x64_mg2": dict(dims=(32, 32, 32, 64), eps=0.5, seed=1, mass=-1.90, nprobes=256, probe_seed=1004,
                            xi=1e-8, block=(4, 4, 4, 4), nv=24, block2=(2, 2, 2, 2), nv2=32, k=256, inner_prec="f16",
                            restart=15, sstep=1, batch=32),
}

PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
