"""Planner formulas and the MLP surrogate in binary64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper Sec. IV: the generic planning instance Y = A X (Eq.
generic_multivector), its flop count (Eq. generic_matvec_flops), the memory
terms (Eqs. planner_workspace, planner_full_cache, planner_partial_cache,
planner_total_memory) and the safety test (Eq. planner_memory_constraint),
waves (Eq. planner_waves), the measured score (Eq. bench_score), the
canonical pair count and cache size (Eq. partial_cache_pairs), the adaptive
block size, and the surrogate network trained on log time with a mean
squared error (Eqs. nn_surrogate, nn_pred_time, nn_loss).  The network here
has the shape this library uses (8 inputs, two hidden layers of 64 ReLU units)
instead of the paper's single tanh layer.
"""
import math

import numpy as np

GiB = 1024 ** 3
MiB = 1024 ** 2


# ---------------------------------------------------------------- Sec. IV-A
def flops_mv(d_out, d_in, R, n_op=1):
    """F_mv = 8 n_op D_out D_in R real operations (Eq. generic_matvec_flops)."""
    return 8 * n_op * d_out * d_in * R


# ---------------------------------------------------------------- Sec. IV-B
def mem_work(r, d_in, R, Bc=8):
    """M_work = r D_in R B_c (Eq. planner_workspace)."""
    return r * d_in * R * Bc


def mem_full(d_out, d_in, n_op=1, p_row=1, Bc=8):
    """M_full = n_op D_out D_in B_c / p_row (Eq. planner_full_cache)."""
    return n_op * d_out * d_in * Bc / p_row


def mem_partial(p_cache, b, n_op=1, Bc=8):
    """M_partial = n_op P_cache b^2 B_c (Eq. planner_partial_cache)."""
    return n_op * p_cache * b * b * Bc


def feasible(m_tot, m_free, alpha=0.9):
    """M_tot <= alpha min_j M_free^(j) (Eq. planner_memory_constraint)."""
    return m_tot <= alpha * min(np.atleast_1d(m_free))


def waves(n_task, groups):
    """W(p) = ceil(N_task / C(p)) (Eq. planner_waves)."""
    return -(-n_task // groups)


def bench_score(n_task, groups, t_mv):
    """S_bench = W(p) t_mv(p) (Eq. bench_score)."""
    return waves(n_task, groups) * t_mv


# ---------------------------------------------------------------- Sec. IV-E/F
def n_pair(n_blk):
    """Canonical Hermitian block pairs n <= m: N_blk (N_blk + 1) / 2."""
    return n_blk * (n_blk + 1) // 2


def p_cache(n_blk, b, m_cache, Bc=8):
    """P_cache = min(N_pair, floor(M_cache / (B_c b^2))) (Eq. partial_cache_pairs)."""
    return min(n_pair(n_blk), int(m_cache // (Bc * b * b)))


def b_target(m_target, Bc=8):
    """b_target ~ sqrt(M_target / B_c) (adaptive block size)."""
    return math.sqrt(m_target / Bc)


def dense_work(D, reuse=1):
    """W_run ~ R_H W_Hpsi with W_Hpsi ~ D^2 (dense-work safety estimate)."""
    return reuse * D * D


# ------------------------------------------------------ surrogate network
def mlp_init(n_in=8, n_hidden=64, seed=0):
    """He-normal initial weights (the paper leaves initialisation open)."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((n_in, n_hidden)) * math.sqrt(2.0 / n_in),
        "b1": np.zeros(n_hidden),
        "W2": rng.standard_normal((n_hidden, n_hidden)) * math.sqrt(2.0 / n_hidden),
        "b2": np.zeros(n_hidden),
        "W3": rng.standard_normal((n_hidden, 1)) * math.sqrt(2.0 / n_hidden),
        "b3": np.zeros(1),
    }


def mlp_forward(p, z):
    """f(z) = relu(relu(z W1 + b1) W2 + b2) W3 + b3; z already normalised."""
    a1 = z @ p["W1"] + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = (h2 @ p["W3"] + p["b3"])[:, 0]
    return y, (z, a1, h1, a2, h2)


def mlp_loss_grad(p, z, target):
    """Mean squared error of log time (Eq. nn_loss) and its gradient."""
    y, (z, a1, h1, a2, h2) = mlp_forward(p, z)
    n = z.shape[0]
    r = y - target
    loss = float(np.mean(r * r))
    gy = (2.0 / n) * r[:, None]
    g = {}
    g["W3"] = h2.T @ gy
    g["b3"] = gy.sum(0)
    gh2 = gy @ p["W3"].T
    ga2 = gh2 * (a2 > 0)
    g["W2"] = h1.T @ ga2
    g["b2"] = ga2.sum(0)
    gh1 = ga2 @ p["W2"].T
    ga1 = gh1 * (a1 > 0)
    g["W1"] = z.T @ ga1
    g["b1"] = ga1.sum(0)
    return loss, g


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of every parameter array in place."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def zscore_fit(x):
    """Componentwise mean and deviation (z = (x - mu) / sigma)."""
    mu = x.mean(0)
    sd = x.std(0)
    sd[sd == 0] = 1.0
    return mu, sd


# ------------------------------------------- analytic planner (Algorithm 1)
# The paper's cost score (Eq. planner_cost_score) leaves the effective
# throughput R_eff and the penalties Pi_cache, Pi_mem undefined.  The reading
# used here makes them a time model of one product built from the runtime
# model of Sec. V: source and contraction overlap (Eq. runtime_overlap), a
# generated entry costs 1/R_gen (Eqs. seed_source_time, analytic_source_time
# with the metadata and latency terms folded into one launch cost), a cached
# entry costs its bytes over the cache bandwidth; the cache penalty becomes
# the fill time, the memory penalty the feasibility test
# (Eq. planner_memory_constraint).  Score = t_fill + reuse t_apply.

PLAN_BLOCKS = (128, 256, 512, 1024, 2048, 4096)
PLAN_MODES = ((0, 0.0), (1, 0.25), (1, 0.5), (1, 0.75), (2, 1.0))   # (strategy, f)
PROCEDURAL, PARTIAL, FULL = 0, 1, 2


def candidates():
    """[(b, strategy, f)]: index = 5 log2(b / 128) + mode."""
    return [(b, st, f) for b in PLAN_BLOCKS for st, f in PLAN_MODES]


def super_edge(D):
    """Work-unit edge 64 se: the largest se in {4, 2} giving >= 45 bands of
    the dimension, else 1."""
    for se in (4, 2):
        if -(-D // (64 * se)) >= 45:
            return 64 * se
    return 64


def uses_matrix_cores(family, strategy, nvec):
    """Binary32 routing: matrix cores for 8+ vectors, or 4+ with every pair
    cached; the procedural sinc-DVR operator always takes its Toeplitz
    kernel."""
    if family == 1 and strategy == PROCEDURAL:
        return False
    return nvec >= 8 or (nvec >= 4 and strategy == FULL)


def vector_blocks(nvec, matrix_cores):
    """Launch blocks of a product: 16 vectors on the matrix cores, else the
    largest of 8, 4, 2, 1 not above what is left."""
    out = []
    r = nvec
    while r > 0:
        k = min(r, 16) if matrix_cores else next(c for c in (8, 4, 2, 1) if c <= r)
        out.append(k)
        r -= k
    return out


def plan_memory(D, nvec, family, b, strategy, f, reuse):
    """(M_op, M_work) bytes: the cache is cached canonical pairs x b^2 x bytes
    per entry (8 complex64, 4 for the real sinc-DVR entries); the workspace
    holds one partial slot per band plus one (per block of 512 columns for
    the procedural sinc-DVR kernel) for the largest vector block (16 on the
    matrix cores), input and output, and with reuse the two Chebyshev
    vectors (complex64 + complex128)."""
    nb = -(-D // b)
    npair = n_pair(nb)
    p = npair if strategy == FULL else int(math.floor(f * npair)) if strategy == PARTIAL else 0
    be = 8.0 if family == 0 else 4.0
    m_op = p * b * b * be
    mc = uses_matrix_cores(family, strategy, nvec)
    blk = 16 if mc else max(vector_blocks(nvec, False)[0], 1)
    if family == 1 and strategy == PROCEDURAL and not mc:
        slots = -(-D // 512)
    else:
        slots = -(-D // super_edge(D)) + 1
    m_work = slots * blk * D * 8.0 + 2.0 * nvec * D * 8.0
    if reuse > 1:
        m_work += nvec * D * (8.0 + 16.0)
    return m_op, m_work


def analytic_time(mm, D, nvec, family, b, strategy, f, reuse):
    """(t_fill, t_apply) seconds of one plan under the machine constants
    mm = {gen_rate: (GUE, DVR) canonical entries/s, dvr_rate: Toeplitz
    elements/s, cache_bw: bytes/s, flop_rate: flop/s, launch_s: s}."""
    m_op, _ = plan_memory(D, nvec, family, b, strategy, f, reuse)
    be = 8.0 if family == 0 else 4.0
    cached = m_op / be                          # cached canonical entries
    canonical = 0.5 * D * (D + 1)               # each applied twice (Hermitian)
    generated = max(0.0, canonical - cached)
    mc = uses_matrix_cores(family, strategy, nvec)
    launches = len(vector_blocks(nvec, mc))
    if family == 1 and strategy == PROCEDURAL and not mc:
        t_src = D * D * nvec / mm["dvr_rate"]   # analytic source, per vector
    else:                                       # every launch regenerates / re-reads
        t_src = launches * (generated / mm["gen_rate"][family] + m_op / mm["cache_bw"])
    t_mv = 8.0 * D * D * nvec / mm["flop_rate"]  # Eq. generic_matvec_flops
    t_apply = mm["launch_s"] + max(t_src, t_mv)  # Eq. runtime_overlap
    t_fill = cached / mm["gen_rate"][family] + m_op / mm["cache_bw"]
    return t_fill, t_apply


def analytic_choice(mm, D, nvec, budget, reuse, family, alpha=0.9):
    """Algorithm 1: the feasible candidate (block not above D except the
    smallest, M_tot <= alpha budget) with the smallest t_fill + reuse t_apply;
    returns (index, score), index None when nothing fits."""
    best, best_score = None, math.inf
    for q, (b, st, f) in enumerate(candidates()):
        if b > D and b != PLAN_BLOCKS[0]:
            continue
        m_op, m_work = plan_memory(D, nvec, family, b, st, f, reuse)
        if not feasible(m_op + m_work, budget, alpha):
            continue
        tf, ta = analytic_time(mm, D, nvec, family, b, st, f, reuse)
        score = tf + reuse * ta
        if score < best_score:
            best, best_score = q, score
    return best, best_score
