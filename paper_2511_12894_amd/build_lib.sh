#!/bin/bash
# Build librf.so for gfx950 from the HIP sources in csrc/ (in-tree).
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
out="${1:-$here/librf.so}"
hipcc --offload-arch=gfx950 -O3 -std=c++17 -fPIC -shared \
  -Xclang -target-feature -Xclang -packed-fp32-ops \
  -Wall -Wno-unused-result \
  -o "$out.tmp" \
  "$here/csrc/api.hip" "$here/csrc/fft.hip" "$here/csrc/spectra.hip" "$here/csrc/recon.hip" "$here/csrc/batch.hip" "$here/csrc/learned.hip" "$here/csrc/factored.hip" "$here/csrc/ols.hip" "$here/csrc/bank.hip"
mv -f "$out.tmp" "$out"
