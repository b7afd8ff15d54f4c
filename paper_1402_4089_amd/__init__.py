"""GPU-resident HMC for Bayesian multinomial regression on MI355X (gfx950)."""
