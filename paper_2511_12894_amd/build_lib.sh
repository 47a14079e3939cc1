#!/bin/bash
# Build librf.so for gfx950 from the HIP sources in csrc/ (in-tree): one object
# per source, compiled in parallel, then linked.
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
out="${1:-$here/librf.so}"
obj="$(mktemp -d "${TMPDIR:-/tmp}/librf_build.XXXXXX")"
trap 'rm -rf "$obj"' EXIT
srcs=(api fft spectra recon batch learned factored ols bank)
pids=()
for s in "${srcs[@]}"; do
  hipcc --offload-arch=gfx950 -O3 -std=c++17 -fPIC -c \
    -Xclang -target-feature -Xclang -packed-fp32-ops \
    -Wall -Wno-unused-result \
    -o "$obj/$s.o" "$here/csrc/$s.hip" &
  pids+=($!)
done
for p in "${pids[@]}"; do wait "$p"; done
objs=()
for s in "${srcs[@]}"; do objs+=("$obj/$s.o"); done
hipcc --offload-arch=gfx950 -shared -fPIC -o "$out.tmp" "${objs[@]}"
mv -f "$out.tmp" "$out"
