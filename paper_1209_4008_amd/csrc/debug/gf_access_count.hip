// gf_access_count.hip -- debug library libgf_debug.so: the site-update
// kernels of libgf compiled with every link-element load and store counted
// (GF_ACCESS_COUNT), to check the RED/BLACK decomposition of Sec. 2 on the
// kernels themselves. In one half-sweep every link of the field must be read
// exactly once and written exactly once (each link belongs to exactly one
// site of the swept parity: U_mu(x) to x, U_mu(y) with y of the other parity
// to y + mu), and the gauge-transformation field of the tracked update must
// be read and written once at each site of the swept parity and not touched
// elsewhere. Since every site reads and writes only its own eight links, the
// counts show that the sites of one launch share no element: the launch has
// no data race. Not part of the product library.
#include "../gf_host.hpp"

#include <type_traits>

// C ABI of the debug library. Returns 0 on success, -1 on bad arguments, -4
// on a HIP error.
//   update: 0 overrelaxation (omega 1.7), 1 heatbath (T 1, seed 1, sweep 0),
//           2 microcanonical, 3 tracked FP32 overrelaxation (needs G, FP32),
//           4 overrelaxation of the maximally Abelian gauge (gauge ignored)
//   U: device field of geom; G: gauge-transformation field (update 3) or NULL
//   reads, writes: zeroed device arrays, one counter per complex element of U
//   (gf_field_bytes / element size); g_reads, g_writes: the same for G
//   (update 3) or NULL
extern "C" int32_t gf_debug_access_count(int32_t update, const gf_geom* g, int32_t gauge,
                                         int32_t parity, int32_t tps, void* U, void* G,
                                         uint32_t* reads, uint32_t* writes, uint32_t* g_reads,
                                         uint32_t* g_writes, void* stream);

namespace {

template <typename T, int NC, int GAUGE, class Upd>
void launch_counted(int tps, void* U, void* Gx, const Lat& L, int parity, const Upd& upd,
                    hipStream_t s) {
  const dim3 grid(blocks_for((uint64_t)L.vh * (uint64_t)tps));
  auto go = [&]<int TPS, bool TRACK>() {
    if constexpr (GAUGE == kMAG)
      hipLaunchKernelGGL((k_mag_half<T, NC, Upd, TPS, kNTNone, TRACK>), grid, dim3(kBlock), 0, s,
                         (v2<T>*)U, L, parity, upd, (v2<T>*)Gx);
    else
      hipLaunchKernelGGL((k_update_half<T, NC, GAUGE, Upd, TPS, kNTNone, TRACK>), grid,
                         dim3(kBlock), 0, s, (v2<T>*)U, L, parity, upd, (v2<T>*)Gx,
                         (const uint8_t*)nullptr);
  };
  auto go_tps = [&]<bool TRACK>() {
    if (tps == 1) go.template operator()<1, TRACK>();
    else if (tps == 2) go.template operator()<2, TRACK>();
    else go.template operator()<4, TRACK>();
  };
  if (Gx) {
    if constexpr (std::is_same<T, float>::value) go_tps.template operator()<true>();
  } else {
    go_tps.template operator()<false>();
  }
}

template <typename T, int NC, int GAUGE>
void dispatch_update(int update, int tps, void* U, void* Gx, const Lat& L, int parity,
                     hipStream_t s) {
  if (update == 1 && GAUGE != kMAG) {
    UpdHB<T> hb;
    hb.temp = (T)1;
    hb.k0 = 1;
    hb.k1 = 0;
    hb.sweep = 0;
    launch_counted<T, NC, GAUGE>(tps, U, nullptr, L, parity, hb, s);
  } else if (update == 2 && GAUGE != kMAG) {
    launch_counted<T, NC, GAUGE>(tps, U, nullptr, L, parity, UpdMicro<T>(), s);
  } else {
    UpdOR<T> o;
    o.omega = (T)1.7;
    launch_counted<T, NC, GAUGE>(tps, U, update == 3 ? Gx : nullptr, L, parity, o, s);
  }
}

}  // namespace

int32_t gf_debug_access_count(int32_t update, const gf_geom* g, int32_t gauge, int32_t parity,
                              int32_t tps, void* U, void* G, uint32_t* reads, uint32_t* writes,
                              uint32_t* g_reads, uint32_t* g_writes, void* stream) {
  if (!geom_ok(g) || update < 0 || update > 4 || (parity != 0 && parity != 1) ||
      (tps != 1 && tps != 2 && tps != 4) || !U || !reads || !writes)
    return -1;
  if (gauge != GF_LANDAU && gauge != GF_COULOMB) return -1;
  if (update == 3 && (g->prec != GF_FP32 || !G || !g_reads || !g_writes)) return -1;
  // sizes as gf_field_bytes and gf_gauge_bytes of libgf give them (this
  // library does not link libgf)
  const Lat L = make_lat(g);
  AccessCount ac = {};
  ac.base[0] = (const char*)U;
  ac.bytes[0] = (size_t)8 * L.vp * (size_t)g->storage * (size_t)g->prec;
  ac.reads[0] = reads;
  ac.writes[0] = writes;
  if (update == 3) {
    ac.base[1] = (const char*)G;
    ac.bytes[1] = (size_t)2 * 6 * L.vp * 2 * sizeof(float);
    ac.reads[1] = g_reads;
    ac.writes[1] = g_writes;
  }
  hipStream_t s = (hipStream_t)stream;
  // synchronous copies, each with the stream drained: the counters are
  // attached exactly for this launch
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(gf_access_count), &ac, sizeof ac) != hipSuccess)
    return -4;
  with_type(g, [&]<typename T, int NC>() {
    if (update == 4)
      dispatch_update<T, NC, kMAG>(update, tps, U, nullptr, L, parity, s);
    else if (gauge == GF_LANDAU)
      dispatch_update<T, NC, kLandau>(update, tps, U, G, L, parity, s);
    else
      dispatch_update<T, NC, kCoulomb>(update, tps, U, G, L, parity, s);
  });
  if (hipGetLastError() != hipSuccess) return -4;
  AccessCount none = {};
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(gf_access_count), &none, sizeof none) != hipSuccess)
    return -4;
  return 0;
}
