"""MI355X-native FP64 ADI-Newton stepper for the thin-film equation (arXiv:1806.10550)."""
