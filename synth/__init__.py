"""Seeded synthetic inputs for the space-VLBI FX correlator.

This package produces station recordings (2-bit samples in the repository's
own Mark5B-style framing) and the job descriptions that go with them.  It is
the only code shared by the CPU oracle and the GPU path, and it holds none of
the correlator's arithmetic: it packs codes, draws noise and simulates what a
station records (a forward model), nothing that unpacks, delays, rotates,
transforms or cross-multiplies.

Modules:
  format   -- frame layout constants and the packer (inverse of unpack)
  job      -- plain job/station description records
  physics  -- exact-physics two-station generator (sky -> station voltages)
  shape    -- shape-only generator (torch, any device) for large configurations
  configs  -- the five workload configurations as concrete parameters
"""
