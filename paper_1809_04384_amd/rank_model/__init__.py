"""Training of the learned rank predictor (data collection on the GPU, training
on the host, compiled-in BF16 weights)."""
