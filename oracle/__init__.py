"""FP64 CPU oracle (test infrastructure only: imported by tests, the smoke check and the CPU baseline)."""
