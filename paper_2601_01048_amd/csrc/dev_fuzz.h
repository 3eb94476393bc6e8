// dev_fuzz.h — the closed-loop fuzzing campaign on the device: mutation of
// corpus entries into a batch of children, bucketed novelty against the
// virgin map, corpus growth and crash signatures.  The check of the children
// between mutation and classification is an ordinary job of the evaluators.
// Part of the device code of libckc; included by kernels.hip only.
#pragma once

namespace ckc {

// SplitMix64 (Steele, Lea and Flood, 2014), counter form: output k of the
// generator started at `seed`.
__device__ __forceinline__ uint64_t fz_draw(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Values a mutation may put in a scalar or an element: 0, 1, -1 and the edges
// of power-of-two ranges.
__constant__ int64_t FZ_VALUES[28] = {
    0, 1, -1, 2, 7, 8, 15, 16, 31, 32, 63, 64, 127, 128, 255, 256, 1023, 1024, 4095, 4096,
    65535, 65536, 2147483647ll, -2147483648ll, 4294967295ll, 4294967296ll, (int64_t)0x8000000000000000ull,
    0x7FFFFFFFFFFFFFFFll};

// AFL's hit-count buckets: 1 | 2 | 3 | 4-7 | 8-15 | 16-31 | 32-127 | 128+,
// one bit each.
__device__ __forceinline__ uint32_t fz_bucket(uint32_t v) {
  if (v == 0) return 0;
  if (v <= 2) return v;
  if (v == 3) return 4;
  // 4-7 -> 8, 8-15 -> 16, 16-31 -> 32, 32-127 -> 64, 128-255 -> 128
  const uint32_t lg = 31u - (uint32_t)__clz(v);  // floor(log2 v), 2..7
  return lg >= 7 ? 128u : (lg >= 5 ? 64u : (8u << (lg - 2)));
}

// One mutation of a child: launch L[6], scalars S[16] (registers), the
// child's elements D in global memory.
__device__ void fz_mutate(const FzArgs& f, uint32_t* L, int64_t* S, int32_t* D, uint64_t u0, uint64_t u1,
                          uint64_t u2) {
  uint32_t ops[3], n = 0;
  if (f.ops & CKC_MUT_LAUNCH) ops[n++] = CKC_MUT_LAUNCH;
  if ((f.ops & CKC_MUT_SCALAR) && f.n_scalars) ops[n++] = CKC_MUT_SCALAR;
  if ((f.ops & CKC_MUT_DATA) && f.n_elems) ops[n++] = CKC_MUT_DATA;
  if (n == 0) return;
  const uint32_t op = ops[u0 % n];
  const uint32_t kind = (uint32_t)((u1 >> 8) & 3u);
  if (op == CKC_MUT_LAUNCH) {
    const uint32_t d = (uint32_t)(u1 % 6);
    const uint64_t old = L[d];
    uint64_t v;
    if (kind == 0) {
      v = old + 1 + u2 % 8;
    } else if (kind == 1) {
      const uint64_t dv = 1 + u2 % 8;
      v = old > dv ? old - dv : 1;
    } else if (kind == 2) {
      v = 1ull << (u2 % 11);
    } else {
      v = 1 + u2 % 256;
    }
    if (v < 1 || v > 0xFFFFFFFFull) return;
    uint32_t M[6];
    for (int q = 0; q < 6; q++) M[q] = q == (int)d ? (uint32_t)v : L[q];
    const uint64_t bs = (uint64_t)M[3] * M[4] * M[5], nb = (uint64_t)M[0] * M[1] * M[2];
    // a child stays inside the campaign's bounds, else the mutation is void
    if (bs <= f.max_block && nb <= 0xFFFFFFFFull && nb * bs <= f.max_threads) L[d] = (uint32_t)v;
  } else if (op == CKC_MUT_SCALAR) {
    const uint32_t k = (uint32_t)(u1 % f.n_scalars);
    uint64_t s = (uint64_t)S[k];
    if (kind == 0) s ^= 1ull << (u2 % 64);
    else if (kind == 1) s += (uint64_t)((int64_t)(u2 % 33) - 16);
    else if (kind == 2) s = (uint64_t)FZ_VALUES[u2 % 28];
    else s = u2;
    S[k] = (int64_t)s;
  } else {
    const uint64_t e = u1 % f.n_elems;
    uint32_t x = (uint32_t)D[e];
    if (kind == 0) x += (uint32_t)((int32_t)(u2 % 33) - 16);
    else if (kind == 1) x = (uint32_t)(uint64_t)FZ_VALUES[u2 % 28];
    else if (kind == 2) x = (uint32_t)u2;
    else x ^= 1u << (u2 % 32);
    D[e] = (int32_t)x;
  }
}

// Workgroup c builds child c of generation g: copy of corpus entry
// r(0) mod size, then 1 + r(1) mod max_stack mutations.  The child's launch
// and scalars go into the job's input c, its elements into its own buffer.
__global__ void __launch_bounds__(256) fuzz_mutate_kernel(FzArgs f, uint64_t g) {
  const uint32_t c = blockIdx.x;
  if (c >= f.batch) return;
  __shared__ uint32_t parent;
  const uint64_t base = (g * f.batch + c) * 64;
  if (threadIdx.x == 0) parent = (uint32_t)(fz_draw(f.seed, base) % f.st->size);
  __syncthreads();
  const uint32_t p = parent;
  int32_t* D = f.child_data + f.n_elems * c;
  const int32_t* src = f.c_data + f.n_elems * p;
  for (uint64_t e = threadIdx.x; e < f.n_elems; e += blockDim.x) D[e] = src[e];
  __syncthreads();
  if (threadIdx.x != 0) return;
  uint32_t L[6];
  int64_t S[MAX_SCALARS];
  for (int q = 0; q < 6; q++) L[q] = f.c_launch[6 * (uint64_t)p + q];
  for (int q = 0; q < MAX_SCALARS; q++) S[q] = f.c_scalars[MAX_SCALARS * (uint64_t)p + q];
  const uint32_t m = 1 + (uint32_t)(fz_draw(f.seed, base + 1) % f.max_stack);
  for (uint32_t j = 0; j < m; j++)
    fz_mutate(f, L, S, D, fz_draw(f.seed, base + 2 + 4 * j), fz_draw(f.seed, base + 3 + 4 * j),
              fz_draw(f.seed, base + 4 + 4 * j));
  for (int q = 0; q < 6; q++) f.in[c].launch[q] = L[q];
  for (int q = 0; q < MAX_SCALARS; q++) f.sc[MAX_SCALARS * (uint64_t)c + q] = S[q];
}

// Workgroup c classifies child c after its check: novel when a site's
// bucketed count shares a bit with the virgin map (as at the generation's
// start; the map is only changed by fuzz_virgin_kernel); its buckets are
// OR-ed into `seen`; every violated (access, kind) keeps the least
// (generation, child) tag.  A map byte is min(255, site count), and only a
// site's byte can be nonzero.
__global__ void __launch_bounds__(256) fuzz_classify_kernel(FzArgs f, uint64_t g) {
  const uint32_t c = blockIdx.x;
  if (c >= f.batch) return;
  const dinput& in = f.in[c];
  const dprog* P = (const dprog*)in.prog;
  const uint16_t* ids = prog_sites(P);
  const uint32_t* cnt = f.counts + in.cnt_base;
  bool nv = false;
  for (uint32_t s = threadIdx.x; s < P->n_map_sites; s += blockDim.x) {
    const uint32_t v = cnt[s] > 255u ? 255u : cnt[s];
    const uint32_t b = fz_bucket(v);
    if (b == 0) continue;
    const uint32_t pos = ids[s];
    if (b & f.virgin[pos]) nv = true;
    atomicOr(&f.seen[pos >> 2], b << (8 * (pos & 3u)));
  }
  const ckc_record* rec = f.recs + in.rec_base;
  bool crash = false;
  const unsigned long long tag = ((unsigned long long)g << 32) | c;
  for (uint32_t a = threadIdx.x; a < P->n_accesses; a += blockDim.x) {
    if (rec[a].count == 0) continue;
    crash = true;
    for (uint32_t k = 0; k < 4; k++)
      if (rec[a].kinds & (1u << k)) atomicMin(&f.sigs[4 * a + k], tag);
  }
  nv = __syncthreads_or(nv);
  crash = __syncthreads_or(crash);
  if (threadIdx.x == 0) {
    f.novel[c] = nv ? 1u : 0u;
    if (nv) atomicAdd((unsigned long long*)&f.st->novel, 1ull);
    if (crash) atomicAdd((unsigned long long*)&f.st->crashes, 1ull);
  }
}

// The generation's buckets leave the virgin map; `seen` is cleared for the
// next generation.  One thread per 32-bit word of the map.
__global__ void __launch_bounds__(256) fuzz_virgin_kernel(FzArgs f) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= 65536 / 4) return;
  const uint32_t s = f.seen[w];
  if (s) {
    uint32_t* v = (uint32_t*)f.virgin + w;
    *v &= ~s;
    f.seen[w] = 0;
  }
}

// One workgroup: novel children, in child order, take the next corpus
// positions while there is room (pos[c], or ~0); their launch, scalars and
// generation are written here, their elements by fuzz_copy_kernel.
__global__ void __launch_bounds__(1024) fuzz_append_kernel(FzArgs f, uint64_t g) {
  __shared__ uint32_t part[1024 / 64];
  __shared__ uint32_t carry;
  const uint32_t t = threadIdx.x;
  const uint32_t size0 = f.st->size;
  if (t == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < f.batch; base += 1024) {
    const uint32_t c = base + t;
    const uint32_t v = c < f.batch ? f.novel[c] : 0u;
    uint32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(incl, o, 64);
      if ((int)(t % 64) >= o) incl += u;
    }
    if (t % 64 == 63) part[t / 64] = incl;
    __syncthreads();
    uint32_t w = 0;
    for (uint32_t q = 0; q < t / 64; q++) w += part[q];
    const uint32_t before = carry + w + incl - v;  // novel children before c
    if (c < f.batch) {
      const uint64_t pos = (uint64_t)size0 + before;
      const bool take = v && pos < f.cap;
      f.pos[c] = take ? (uint32_t)pos : ~0u;
      if (take) {
        for (int q = 0; q < 6; q++) f.c_launch[6 * pos + q] = f.in[c].launch[q];
        for (int q = 0; q < MAX_SCALARS; q++) f.c_scalars[MAX_SCALARS * pos + q] = f.sc[MAX_SCALARS * (uint64_t)c + q];
        f.c_gen[pos] = (uint32_t)g;
      }
    }
    __syncthreads();
    if (t == 1023) carry = carry + w + incl;
    __syncthreads();
  }
  if (t == 0) {
    const uint64_t grown = (uint64_t)size0 + carry;
    f.st->size = (uint32_t)(grown < f.cap ? grown : f.cap);
    f.st->execs += f.batch;
    f.st->generations += 1;
  }
}

// Workgroup c copies the elements of an appended child into its corpus entry.
__global__ void __launch_bounds__(256) fuzz_copy_kernel(FzArgs f) {
  const uint32_t c = blockIdx.x;
  if (c >= f.batch || f.n_elems == 0) return;
  const uint32_t pos = f.pos[c];
  if (pos == ~0u) return;
  const int32_t* src = f.child_data + f.n_elems * c;
  int32_t* dst = f.c_data + f.n_elems * pos;
  for (uint64_t e = threadIdx.x; e < f.n_elems; e += blockDim.x) dst[e] = src[e];
}

}  // namespace ckc
