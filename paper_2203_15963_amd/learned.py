"""Learned step proposals: log the plain integrator, train the network on
the GPU, install it.  Orchestration of library calls only (every step runs
in the library's kernels)."""
from paper_2203_15963_amd import synth


def train_step_model(ctx, n_images=128, n=32, seed=3, epochs=4, batch=16384, lr=2e-3, val_frac=0.1,
                     capacity=None):
    """Returns (model tensor, losses [epochs][2], number of logged steps,
    records).  A val_frac share of the records, drawn by a pseudo-random
    order of the rows, is held out."""
    wl = synth.steplog_workload(n_images=n_images, n=n, seed=seed)
    if capacity is None:
        capacity = n_images * n * n * 400
    rec, n_steps = ctx.steplog(wl["images"], wl["integrator"], capacity)
    n_val = int(val_frac * rec.shape[0]) // 64 * 64
    model = ctx.mlp_init(rec, seed=seed)
    losses = ctx.mlp_train(rec, model, epochs=epochs, batch=batch, lr=lr, seed=seed, n_val=n_val)
    return model, losses, n_steps, rec
