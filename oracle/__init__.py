"""Oracle package: plain FP64 CPU statement of the HISQ solve path (test infrastructure only)."""
